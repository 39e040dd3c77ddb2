"""Pins of the oracle's time-periodic problem u(0) = u(T) (section 3,
eqs. chap4_equationLinearSystemODEPeriodic and chap4_circulantMatrix: the
block system with the circulant coupling, slab 1 coupled to slab N) against
what the mathematics fixes:

* the operator equals the dense circulant matrix I (x) A + U~_N (x) N built
  from the closed-form slab matrices (forward and transposed);
* the exact solve equals a dense solve of that matrix, and its residual
  vanishes at N = 1000;
* a constant load reproduces the exact periodic solution u = f0 / lambda
  (polynomials of degree <= p are reproduced exactly);
* one periodic two-grid cycle (coarse level N/2 solved exactly) is, column
  by column, the dense two-grid propagator of the circulant system, and its
  spectral radius is the Fourier estimate of Theorem chap4_theorem4, which is
  exact for periodic problems;
* V and W cycles over several levels equal the dense recursive propagator
  (eq. chap4_errorTwoGridCycle applied recursively) of the circulant levels;
* the measured contraction of the two-grid cycle from a random start lies
  under the estimate (up to the 1e-5 window bias of the non-periodic pin)
  and above 0.9 of it.
All CPU (not gpu)."""
import numpy as np
import pytest

from oracle import analysis as an
from oracle import core


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("trans", [False, True])
def test_periodic_operator_is_the_circulant_matrix(p, trans):
    rng = np.random.default_rng(300 + p)
    N, tau, lam = 16, 0.37, 1.9
    u = rng.standard_normal(N * (p + 1))
    L = an.dense_L(p, N, tau, lam, periodic=True)
    ref = (L.T if trans else L) @ u
    out = core.apply(p, tau, lam, u, trans=trans, periodic=True)
    assert np.max(np.abs(out - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the non-periodic operator differs exactly in the wrap-around coupling
    Lnp = an.dense_L(p, N, tau, lam, periodic=False)
    assert not np.allclose(L, Lnp)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("z", [1e-3, 0.5, 40.0])
def test_periodic_direct_solve(p, trans, z):
    rng = np.random.default_rng(310 + p)
    N, lam = 32, 1.0
    f = rng.standard_normal(N * (p + 1))
    L = an.dense_L(p, N, z, lam, periodic=True)
    ref = np.linalg.solve(L.T if trans else L, f)
    u = core.direct(p, z, lam, f, trans=trans, periodic=True)
    assert np.max(np.abs(u - ref)) <= 1e-11 * np.max(np.abs(ref))
    # a longer one: the residual of the circulant system vanishes
    N2 = 1000
    f2 = rng.standard_normal(N2 * (p + 1))
    u2 = core.direct(p, z, lam, f2, trans=trans, periodic=True)
    r2 = core.residual(p, z, lam, f2, u2, trans=trans, periodic=True)
    assert np.max(np.abs(r2)) <= 1e-12 * max(np.max(np.abs(f2)), np.max(np.abs(u2)))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("lam", [0.3, 1.0, 25.0])
def test_periodic_constant_load(p, lam):
    """u' + lambda u = f0 with u(0) = u(T) has the solution f0 / lambda; its
    load vector is f_n = tau f0 e_0 (int P_k = 0 for k >= 1), and the DG
    solution is that constant: coefficient 0 equal to f0 / lambda, the others
    zero."""
    N, T, f0 = 64, 3.0, 2.5
    tau = T / N
    P = p + 1
    f = np.zeros(N * P)
    f[0::P] = tau * f0
    u = core.direct(p, tau, lam, f, periodic=True)
    ref = np.zeros(N * P)
    ref[0::P] = f0 / lam
    assert np.max(np.abs(u - ref)) <= 1e-13 * f0 / lam


def _cycle_matrix(p, N, T, lam, opts, trans=False):
    """The oracle's one-cycle error propagator on f = 0, column by column."""
    n = N * (p + 1)
    M = np.empty((n, n))
    f = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        M[:, i] = core.cycles(p, T, lam, f, e, 1, opts, trans=trans, periodic=True)
    return M


@pytest.mark.parametrize("p", [0, 1, 2])
@pytest.mark.parametrize("z", [1e-3, 0.7, 6.0])
@pytest.mark.parametrize("nu", [1, 2])
def test_periodic_two_grid_operator_and_symbol(p, z, nu):
    N = 32
    om = an.omega_opt(an.alpha_of(p, z))
    opts = core.Opts(nu1=nu, nu2=nu, gamma=1, n_coarse=N // 2)
    M = _cycle_matrix(p, N, z * N, 1.0, opts)
    D = an.dense_two_grid(p, N, z, nu, nu, om, periodic=True)
    assert np.max(np.abs(M - D)) <= 1e-12 * max(1.0, np.max(np.abs(D)))
    rho = float(np.max(np.abs(np.linalg.eigvals(M))))
    est = an.two_grid_rho(p, z, nu, nu, om, N=N)
    assert rho == pytest.approx(est, rel=1e-8, abs=1e-13)


@pytest.mark.parametrize("p", [0, 1, 3])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("trans", [False, True])
def test_periodic_multilevel_cycle(p, gamma, trans):
    N, T, lam = 32, 5.0, 1.3
    opts = core.Opts(nu1=2, nu2=1, gamma=gamma, n_coarse=2)
    M = _cycle_matrix(p, N, T, lam, opts, trans=trans)
    D = an.dense_cycle(p, N, T, lam, 2, 1, gamma, n_coarse=2, trans=trans, periodic=True)
    assert np.max(np.abs(M - D)) <= 1e-13 * max(1.0, np.max(np.abs(D)))


@pytest.mark.parametrize("p,z,nu", [(0, 1e-3, 1), (1, 1e-3, 1), (1, 1.0, 2), (3, 0.1, 1),
                                    (5, 1e-2, 1)])
def test_periodic_measured_contraction(p, z, nu):
    N = 1024
    P = p + 1
    rng = np.random.default_rng(200 + p)
    u = rng.uniform(0.0, 1.0, N * P)
    f = np.zeros_like(u)
    opts = core.Opts(nu1=nu, nu2=nu, gamma=1, n_coarse=N // 2)
    r = [np.linalg.norm(core.residual(p, z, 1.0, f, u, periodic=True))]
    while len(r) < 40 and r[-1] > 1e-200 * r[0]:
        u = core.cycles(p, z * N, 1.0, f, u, 1, opts, periodic=True)
        r.append(np.linalg.norm(core.residual(p, z, 1.0, f, u, periodic=True)))
    K = len(r) - 1
    tail = (r[K] / r[K // 2]) ** (1.0 / (K - K // 2))
    est = an.two_grid_rho(p, z, nu, nu, N=N)
    assert 0.9 * est <= tail <= (1.0 + 1e-5) * est


@pytest.mark.parametrize("p", [0, 2])
def test_periodic_solve_converges_to_direct(p):
    rng = np.random.default_rng(320 + p)
    N, T, lam = 512, 20.0, 0.8
    f = rng.standard_normal(N * (p + 1)) * 0.01
    u, k, rr, _ = core.solve_folded(p, T, lam, f, rtol=1e-10, periodic=True)
    ud = core.direct(p, T / N, lam, f, periodic=True)
    assert rr <= 1e-10 and k <= 20
    assert np.max(np.abs(u - ud)) <= 1e-8 * np.max(np.abs(ud))
