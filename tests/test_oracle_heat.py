"""Pins of the oracle's space-time heat equation (section 6: the time
multigrid applied to u_t = u_xx + f; here on (0,1) with u = 0 at both ends,
second-order finite differences on nx interior points, DG in time), CPU
only:

* the operator equals the dense Kronecker form
  I_x (x) (I_N (x) K - U_N (x) N) + L_h (x) I_N (x) M built from the
  closed-form slab matrices and L_h = tridiag(-1, 2, -1) / h^2;
* the orthonormal sine transform S (S L_h S = diag(lambda_j),
  lambda_j = (4/h^2) sin^2(j pi h / 2)) decouples the problem into the ODEs
  u' + lambda_j u = f_j: the exact solve, and whole V and W cycles with a
  damping that is the same for every mode, equal S applied to the pinned
  ODE oracle's solves and cycles mode by mode;
* the per-level damping is Lemma chap4_lemma7's at lambda_1 tau_l;
* the discrete sine mode u0 = sin(pi x) decays by exactly alpha(lambda_1 tau)
  per slab (the end values of the (p, p+1) Pade step);
* the multigrid solve converges to the direct solve."""
import numpy as np
import pytest

from oracle import analysis as an
from oracle import core


def sine(nx):
    h = 1.0 / (nx + 1)
    j = np.arange(1, nx + 1)
    S = np.sqrt(2.0 * h) * np.sin(np.pi * np.outer(j, j) * h)
    lam = 4.0 / h ** 2 * np.sin(j * np.pi * h / 2.0) ** 2
    return S, lam


def Lh(nx):
    h = 1.0 / (nx + 1)
    return (2.0 * np.eye(nx) - np.eye(nx, k=1) - np.eye(nx, k=-1)) / h ** 2


def to_modes(S, a, nx, N, P):
    """[point][slab][k] -> [mode][slab][k] with the sine transform."""
    return (S @ a.reshape(nx, N * P)).reshape(-1)


def test_sine_transform_diagonalises():
    S, lam = sine(9)
    assert np.allclose(S @ S, np.eye(9), atol=1e-14)
    assert np.allclose(S @ Lh(9) @ S, np.diag(lam), atol=1e-10)


@pytest.mark.parametrize("p", [0, 1, 3])
def test_heat_operator_is_the_kronecker_form(p):
    rng = np.random.default_rng(400 + p)
    nx, N, tau = 7, 6, 0.05
    P = p + 1
    K, M, Nm, _ = an.slab_closed_form(p, tau, 1.0)
    Lt = np.kron(np.eye(N), K) - np.kron(np.eye(N, k=-1), Nm)
    L = np.kron(np.eye(nx), Lt) + np.kron(Lh(nx), np.kron(np.eye(N), M))
    u = rng.standard_normal(nx * N * P)
    out = core.heat_apply(p, nx, tau, u)
    assert np.max(np.abs(out - L @ u)) <= 1e-13 * np.max(np.abs(L @ u))


@pytest.mark.parametrize("p", [0, 1, 2, 4])
@pytest.mark.parametrize("nx,N,T", [(7, 32, 0.3), (15, 64, 2.0)])
def test_heat_direct_decouples(p, nx, N, T):
    rng = np.random.default_rng(410 + p)
    P = p + 1
    S, lam = sine(nx)
    f = rng.standard_normal(nx * N * P)
    u = core.heat_direct(p, nx, T / N, f)
    fh = to_modes(S, f, nx, N, P).reshape(nx, N * P)
    uh = np.stack([core.direct(p, T / N, lam[j], fh[j]) for j in range(nx)])
    ref = to_modes(S, uh.reshape(-1), nx, N, P)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [0, 1, 3])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("nu", [(2, 2), (1, 3)])
def test_heat_cycle_decouples(p, gamma, nu):
    """With one damping for all modes (a fixed omega), one heat cycle is the
    sine transform of the ODE cycles of every mode."""
    rng = np.random.default_rng(420 + p)
    nx, N, T = 7, 64, 0.8
    P = p + 1
    S, lam = sine(nx)
    opts = core.Opts(nu1=nu[0], nu2=nu[1], gamma=gamma, n_coarse=2, omega_mode=1, omega=0.6)
    f, u = rng.standard_normal(nx * N * P), rng.standard_normal(nx * N * P)
    out = core.heat_cycles(p, nx, T, f, u, 2, opts)
    fh = to_modes(S, f, nx, N, P).reshape(nx, N * P)
    uh = to_modes(S, u, nx, N, P).reshape(nx, N * P)
    oh = np.stack([core.cycles(p, T, lam[j], fh[j], uh[j], 2, opts) for j in range(nx)])
    ref = to_modes(S, oh.reshape(-1), nx, N, P)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [0, 1, 3, 5])
def test_heat_level_damping(p):
    nx, N, T = 31, 256, 1.5
    w = core.heat_levels(p, nx, N, T)
    h = 1.0 / (nx + 1)
    lam1 = 4.0 / h ** 2 * np.sin(np.pi * h / 2.0) ** 2
    for l, wl in enumerate(w):
        tau = T / (N >> l)
        assert wl == pytest.approx(an.omega_opt(an.alpha_of(p, lam1 * tau)), rel=1e-13)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_heat_sine_mode_decay(p):
    """u0 = sin(pi x_i), f = 0: the discrete sine mode is an eigenvector of
    L_h, so the end values decay by alpha(lambda_1 tau) per slab exactly."""
    nx, N, T = 15, 40, 0.2
    P = p + 1
    h = 1.0 / (nx + 1)
    x = h * np.arange(1, nx + 1)
    u0 = np.sin(np.pi * x)
    lam1 = 4.0 / h ** 2 * np.sin(np.pi * h / 2.0) ** 2
    f = core.heat_fold(p, nx, u0, np.zeros(nx * N * P))
    u = core.heat_direct(p, nx, T / N, f).reshape(nx, N, P)
    w = u.sum(axis=2)                       # end values u_n(t_n^-) at every point
    a = an.alpha_of(p, lam1 * T / N)
    ref = np.outer(u0, a ** np.arange(1, N + 1))
    assert np.max(np.abs(w - ref)) <= 1e-13


@pytest.mark.parametrize("p", [0, 1, 3])
@pytest.mark.parametrize("gamma", [1, 2])
def test_heat_solve_converges(p, gamma):
    rng = np.random.default_rng(430 + p)
    nx, N, T = 15, 128, 1.0
    P = p + 1
    f = rng.standard_normal(nx * N * P) * 0.01
    u, k, rr, hist = core.heat_solve_folded(p, nx, T, f, opts=core.Opts(gamma=gamma))
    ud = core.heat_direct(p, nx, T / N, f)
    assert rr <= 1e-10 and k <= 20
    assert np.all(np.diff(np.log(hist)) < 0)
    assert np.max(np.abs(u - ud)) <= 1e-8 * np.max(np.abs(ud))
