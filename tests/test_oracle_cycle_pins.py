"""Pins of the oracle's multi-level cycle (V and W) against the dense
recursive error propagator.

The cycle is the two-grid method of eq. chap4_errorTwoGridCycle (section 3)
applied recursively: on a level with a coarser one, nu1 damped block Jacobi
sweeps, the residual restricted, gamma cycles of the next level from zero on
the coarse error equation (an exact solve on the coarsest level), the
prolongated correction, nu2 sweeps.  Its error propagator is therefore

    M_l = S_l^nu2 (I - P (I - M_{l+1}^gamma) L_{l+1}^{-1} R L_l) S_l^nu1,
    M_coarsest = 0,

and one cycle maps u to M_0 u + (I - M_0) L^{-1} f.  analysis.dense_cycle
builds M_0 from the closed-form slab matrices and the Legendre re-expansion
of the transfers; the C oracle builds everything by quadrature and runs the
recursion on vectors.  A cycle that ignores gamma, restarts the coarse error
between the gamma visits, swaps nu1 and nu2, uses the wrong level's damping
or the wrong coarse operator fails these tests (the last test checks that the
V and W propagators differ by far more than the tolerance, so the pin sees
gamma at all).
"""
import numpy as np
import pytest

from oracle import analysis as an
from oracle import core


def _oracle_matrix(p, N, T, lam, opts, trans):
    """Columns of the oracle's one-cycle map on L u = 0 (f = 0): M_0 e_i."""
    n = N * (p + 1)
    f = np.zeros(n)
    M = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, i] = core.cycles(p, T, lam, f, e, 1, opts, trans=trans)
    return M


CASES = [
    # (N, n_coarse, nu1, nu2, T, lam): 4 to 5 levels, uneven sweeps
    (16, 2, 2, 1, 3.0, 2.0),
    (32, 2, 1, 3, 10.0, 1.0),
    (32, 4, 2, 2, 0.5, 40.0),
    (8, 1, 3, 2, 2.0, 0.3),
]


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_cycle_error_propagator(p, gamma, trans, case):
    """The oracle's cycle equals M_0 column by column (1e-13 of max|M_0|)."""
    N, nc, nu1, nu2, T, lam = case
    opts = core.Opts(nu1=nu1, nu2=nu2, gamma=gamma, n_coarse=nc)
    Md = an.dense_cycle(p, N, T, lam, nu1, nu2, gamma, n_coarse=nc, trans=trans)
    Mo = _oracle_matrix(p, N, T, lam, opts, trans)
    assert np.max(np.abs(Mo - Md)) <= 1e-13 * max(np.max(np.abs(Md)), 1e-3)


@pytest.mark.parametrize("p", [1, 3])
@pytest.mark.parametrize("gamma", [1, 2])
def test_cycle_affine_part_and_fixed_damping(p, gamma):
    """From u = 0 one cycle gives (I - M_0) L^{-1} f; with the fixed damping
    omega = 1/2 (section 3.2) as well."""
    N, T, lam = 32, 4.0, 1.5
    n = N * (p + 1)
    rng = np.random.default_rng(7 + p)
    f = rng.standard_normal(n)
    L = an.dense_L(p, N, T / N, lam)
    for omega in (None, 0.5):
        opts = core.Opts(gamma=gamma, omega_mode=0 if omega is None else 1,
                         omega=0.5 if omega is None else omega)
        Md = an.dense_cycle(p, N, T, lam, 2, 2, gamma, omega=omega)
        ref = (np.eye(n) - Md) @ np.linalg.solve(L, f)
        u = core.cycles(p, T, lam, f, np.zeros(n), 1, opts)
        assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [0, 2])
def test_pin_separates_v_from_w(p):
    """With four or more levels the V and W propagators differ by many
    orders of magnitude more than the tolerance above."""
    N, T, lam = 32, 10.0, 1.0
    Mv = an.dense_cycle(p, N, T, lam, 2, 2, 1)
    Mw = an.dense_cycle(p, N, T, lam, 2, 2, 2)
    assert np.max(np.abs(Mv - Mw)) >= 1e6 * 1e-13 * np.max(np.abs(Mv))


# FP32-inner cycle of the defect correction.  Every FP32 operation rounds
# with a relative error of at most u32 = 2^-24.  The cycle is a fixed
# sequence of contractive steps (sweeps with |1 - omega| + |h| <= 1, exact
# transfers, residuals computed in FP64), so its rounding errors add up to a
# small multiple of u32 times the size of the exact correction
# x = L^{-1} r.  The stated bound is 32 u32 ||x||_inf (~1.9e-6); measured:
# about 1.4 u32.
U32 = 2.0 ** -24
MIXED_BOUND = 32 * U32


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("lb64", [-1, 2])
@pytest.mark.parametrize("z", [1e-3, 0.5, 30.0])
def test_mixed_cycle_against_fp64_propagator(p, gamma, lb64, z):
    """One FP32-inner cycle from zero equals (I - M_0) L^{-1} r up to the FP32
    rounding bound above, with the levels from lb64 on computed in FP64 (-1:
    the coarsest only)."""
    N = 32
    T = z * N
    lam = 1.0
    n = N * (p + 1)
    rng = np.random.default_rng(11 + p)
    r = rng.standard_normal(n)
    r32 = r.astype(np.float32).astype(np.float64)
    L = an.dense_L(p, N, T / N, lam)
    x = np.linalg.solve(L, r32)
    Md = an.dense_cycle(p, N, T, lam, 2, 2, gamma)
    ref = (np.eye(n) - Md) @ x
    e = core.cycle_mixed(p, T, lam, r, core.Opts(gamma=gamma), lb64=lb64)
    err = np.max(np.abs(e - ref)) / np.max(np.abs(x))
    assert err <= MIXED_BOUND, err
    # and the rounding is really FP32 (not an FP64 cycle in disguise)
    e64 = core.cycles(p, T, lam, r32, np.zeros(n), 1, core.Opts(gamma=gamma))
    assert np.max(np.abs(e - e64)) > 1e-12 * np.max(np.abs(x))
