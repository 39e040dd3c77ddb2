"""Writes two_grid_rho.json: the two-grid contraction estimate (the largest
spectral radius of the Fourier symbol over the low frequencies, Theorem
chap4_theorem4; per-level optimal damping) for the cases the GPU replay of
the section 4.2 convergence study checks.  Calls the oracle only.

    python tests/golden/make_two_grid_rho.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import analysis as an  # noqa: E402

N = 1024
CASES = [(p, z, nu) for p in range(6) for z in (1e-3, 1.0, 40.0) for nu in (1, 2, 5)]


def main():
    out = {"N": N, "cases": []}
    for p, z, nu in CASES:
        out["cases"].append({"p": p, "z": z, "nu": nu, "rho": an.two_grid_rho(p, z, nu, nu, N=N)})
    with open(os.path.join(HERE, "two_grid_rho.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
