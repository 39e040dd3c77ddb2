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
# the grid of the section 4.2 figures: tau = z in 10^-6 .. 10^6 (13 points),
# p = 0..5, nu1 = nu2 in {1, 2, 5}
ZS = [10.0 ** e for e in range(-6, 7)]
CASES = [(p, z, nu) for p in range(6) for z in ZS for nu in (1, 2, 5)]


def main():
    out = {"N": N, "cases": []}
    for p, z, nu in CASES:
        out["cases"].append({"p": p, "z": z, "nu": nu, "rho": an.two_grid_rho(p, z, nu, nu, N=N)})
    with open(os.path.join(HERE, "two_grid_rho.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
