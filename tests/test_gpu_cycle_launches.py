"""GPU parity of the cycles' launch forms: the dense bottom operator
(tmg_set_dense_bottom, V and W) and the W-cycle's fused streaming legs.

The gamma visits that a cycle (eq. chap4_errorTwoGridCycle of section 3,
applied recursively with the exact solve on the coarsest level) makes of a
level from a zero iterate are one linear map of that level's right-hand
side; the library tabulates it once per schedule and tables and applies it
as a matrix.  The cycles are then the oracle's W-cycles up to the rounding of
the matrix-vector product (its sums run in another order than the
recursion's), so the bars are those of the other FP64 cycle tests: 1e-12
against the oracle, for cycles from identical inputs and for converged
solves with the same number of cycles.

The streaming levels of one instance's W-cycle run in fused launches (the
first visit's up leg with the second visit's down leg, and each first
visit's down leg with the level above's launch) when the schedule has
two-level launches on; every kernel computes what the one-level legs
compute, in the same order, so with them off the iterates must be equal to
the last bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
TOL = 1e-12


def B():
    from paper_1409_5254_amd import binding
    return binding


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def bottom_max(P):
    """Largest level of the bottom kernel (its work-group's slabs)."""
    return (256 if P >= 5 else 512) * {1: 8, 2: 4}.get(P, 2)


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("log2cap", [3, 5, 7, 9])
def test_dense_cycles_match_oracle(p, log2cap, gamma):
    """Three V- or W-cycles from a random start (tmg_vcycle) with the dense
    bottom operator at a bottom level of 2^log2cap slabs, and with the
    recursion at every visit, both against the oracle's cycles."""
    P = p + 1
    cap = 1 << log2cap
    if cap > bottom_max(P) or cap * P > 4096:
        pytest.skip("bottom level larger than the bottom kernel's or the dense operator's")
    rng = np.random.default_rng(300 + 10 * p + log2cap)
    N, T, lam, u0 = 4096, 10.0, 1.3, 0.5
    f, u = rng.standard_normal(N * P), rng.standard_normal(N * P)
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, core.Opts(gamma=gamma))
    out = {}
    for on in (True, False):
        s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
        s.set_schedule(cap, pairs=True)
        s.set_dense_bottom(on)
        du = dev(u)
        for _ in range(3):
            s.vcycle(dev(f), dev([u0]), du)
        out[on] = host(du)
        s.close()
        assert relerr(out[on], ref) <= TOL, (on, relerr(out[on], ref))
    assert relerr(out[True], out[False]) <= TOL


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("p,log2n,cap", [(0, 16, 4096), (1, 16, 2048), (3, 15, 1024),
                                         (3, 14, 1024), (5, 14, 512), (2, 13, 64)])
def test_dense_solve_matches_oracle(p, log2n, cap, gamma):
    """V(2,2) and W(2,2) solves to 1e-10 with the dense bottom operator at its
    largest sizes (4096 unknowns) and a small one: the oracle's cycle count
    and its solution at 1e-12."""
    P = p + 1
    rng = np.random.default_rng(500 + p + log2n)
    N = 1 << log2n
    T, lam, u0 = 1000.0 * N / (1 << 22), 1.0, 1.0
    f = rng.standard_normal(N * P)
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
    s.set_schedule(cap, pairs=True, direct=True)
    res = s.solve(dev(f), dev([u0]), rtol=1e-10, max_cycles=60)
    u = host(res.u)
    s.close()
    uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(gamma=gamma))
    assert res.status == 0 and res.cycles[0] == k, (res.status, res.cycles, k)
    assert relerr(u, uo) <= TOL


def test_dense_rebuilt_after_lambda_and_schedule():
    """The operator follows the tables and the schedule: a new lambda (set
    on the device) and then a new bottom level, each followed by W-cycles
    against the oracle's for the same problem; graphs captured before each
    change are replayed after it."""
    p, N, T, u0 = 2, 4096, 10.0, 0.5
    P = p + 1
    rng = np.random.default_rng(77)
    f, u = rng.standard_normal(N * P), rng.standard_normal(N * P)
    s = B().Solver([N], [T], [1.3], p=p, gamma=2)
    s.set_schedule(256, pairs=True)
    for lam, cap in ((1.3, 256), (40.0, 256), (40.0, 64), (0.01, 64)):
        if cap != 256:
            s.set_schedule(cap, pairs=True)
        s.set_lambda(dev([lam]))
        res = s.solve(dev(f), dev([u0]), rtol=1e-10, max_cycles=60)
        uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(gamma=2))
        assert res.status == 0 and res.cycles[0] == k, (lam, cap, res.cycles, k)
        assert relerr(host(res.u), uo) <= TOL, (lam, cap)
        du = dev(u)
        s.vcycle(dev(f), dev([u0]), du)
        ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 1, core.Opts(gamma=2))
        assert relerr(host(du), ref) <= TOL, (lam, cap)
    s.close()


def test_dense_batches_and_adjoint():
    """A batch runs the recursion (the operator is one instance's); one
    instance's adjoint solve applies the transposed system's operator (its
    columns are the backward-in-time visits): a two-instance batch and the
    adjoint W solve of one instance against the oracle."""
    p, N, T = 1, 2048, 10.0
    P = p + 1
    rng = np.random.default_rng(78)
    fs = [rng.standard_normal(N * P) for _ in range(2)]
    lams = [1.0, 7.0]
    s = B().Solver([N, N], [T, T], lams, p=p, gamma=2)
    s.set_schedule(128, pairs=True)
    res = s.solve(dev(np.concatenate(fs)), dev([0.5, 0.25]), rtol=1e-10, max_cycles=60)
    u = host(res.u)
    s.close()
    for j in range(2):
        uo, k, _, _ = core.solve(p, T, lams[j], [0.5, 0.25][j], fs[j], opts=core.Opts(gamma=2))
        assert res.cycles[j] == k
        assert relerr(u[j * N * P:(j + 1) * N * P], uo) <= TOL
    s = B().Solver([N], [T], [1.0], p=p, gamma=2)
    s.set_schedule(128, pairs=True)
    fw = s.solve(dev(fs[0]), dev([0.5]), rtol=1e-10, max_cycles=60)
    z, _, _, cyc, _, st = s.adjoint_solve(dev(fs[1]), u=fw.u, rtol=1e-10, max_cycles=60)
    z = host(z)
    s.close()
    zo, kz, _, _ = core.solve_folded(p, T, 1.0, fs[1], rtol=1e-10, trans=True,
                                     opts=core.Opts(gamma=2))
    assert st == 0 and cyc[0] == kz
    assert relerr(z, zo) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("nu", [(2, 2), (1, 0), (0, 3), (3, 1)])
@pytest.mark.parametrize("dense", [True, False])
def test_fused_w_legs_bitwise(p, nu, dense):
    """Three W-cycles of one instance with the fused streaming launches and
    with one-level legs, bitwise equal, and both equal to the oracle's
    cycles at 1e-12 (N = 2^13: eight streaming levels above a bottom level
    of 32 slabs, ragged tiles at every level)."""
    P = p + 1
    nu1, nu2 = nu
    rng = np.random.default_rng(900 + 10 * p + nu1 * 4 + nu2)
    N, T, lam, u0 = 8192, 20.0, 0.7, 0.5
    f, u = rng.standard_normal(N * P), rng.standard_normal(N * P)
    out = {}
    for pairs in (True, False):
        s = B().Solver([N], [T], [lam], p=p, gamma=2, nu1=nu1, nu2=nu2)
        s.set_schedule(32, pairs=pairs)
        s.set_dense_bottom(dense)
        du = dev(u)
        for _ in range(3):
            s.vcycle(dev(f), dev([u0]), du)
        out[pairs] = host(du)
        s.close()
    assert np.array_equal(out[True], out[False])
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, core.Opts(gamma=2, nu1=nu1, nu2=nu2))
    assert relerr(out[True], ref) <= TOL


@pytest.mark.parametrize("p", [1, 3])
def test_fused_w_solve_and_adjoint(p):
    """A W(2,2) solve and the adjoint solve of one instance with the fused
    launches (N = 2^14, bottom level 64 slabs) against the oracle: the same
    cycle counts, solutions at 1e-12."""
    P = p + 1
    rng = np.random.default_rng(950 + p)
    N, T, lam, u0 = 16384, 40.0, 1.1, 0.3
    f, g = rng.standard_normal(N * P), rng.standard_normal(N * P)
    s = B().Solver([N], [T], [lam], p=p, gamma=2)
    s.set_schedule(64, pairs=True)
    res = s.solve(dev(f), dev([u0]), rtol=1e-10, max_cycles=60)
    z, _, _, cyc, _, st = s.adjoint_solve(dev(g), u=res.u, rtol=1e-10, max_cycles=60)
    u, z = host(res.u), host(z)
    s.close()
    uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(gamma=2))
    assert res.status == 0 and res.cycles[0] == k
    assert relerr(u, uo) <= TOL
    zo, kz, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-10, trans=True, opts=core.Opts(gamma=2))
    assert st == 0 and cyc[0] == kz
    assert relerr(z, zo) <= TOL


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("opts", [dict(n_coarse=1), dict(n_coarse=4), dict(nu1=1, nu2=3),
                                  dict(nu1=3, nu2=0), dict(omega_mode=1, omega=0.5)])
@pytest.mark.parametrize("p", [0, 2, 5])
def test_dense_bottom_options(p, opts, gamma):
    """The dense bottom operator under the other options: coarsest levels
    of 1 and 4 slabs, uneven sweep counts, the fixed damping 1/2.  Three
    cycles (tmg_vcycle) and a solve against the oracle at 1e-12; the
    operator on and off give the same cycle count."""
    P = p + 1
    nc = opts.get("n_coarse", 2)
    N = 1024 * nc
    rng = np.random.default_rng(1300 + p + 7 * gamma + len(str(opts)))
    T, lam, u0 = 6.0, 1.7, 0.3
    f, u = rng.standard_normal(N * P), rng.standard_normal(N * P)
    oo = core.Opts(gamma=gamma, **opts)
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, oo)
    uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=oo)
    cyc = {}
    for on in (True, False):
        s = B().Solver([N], [T], [lam], p=p, gamma=gamma, **opts)
        s.set_schedule(min(64 * nc, 512), pairs=True)
        s.set_dense_bottom(on)
        du = dev(u)
        for _ in range(3):
            s.vcycle(dev(f), dev([u0]), du)
        assert relerr(host(du), ref) <= TOL, (on, relerr(host(du), ref))
        res = s.solve(dev(f), dev([u0]), rtol=1e-10, max_cycles=80)
        assert res.status == 0 and res.cycles[0] == k, (on, res.cycles, k)
        assert relerr(host(res.u), uo) <= TOL
        cyc[on] = res.cycles[0]
        s.close()
    assert cyc[True] == cyc[False]


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("p", [0, 1, 3, 5, 6, 10])
def test_dense_adjoint_on_off(p, gamma):
    """The adjoint solve of one instance with the transposed operator and
    with the recursion: the same cycle count, both at 1e-12 of the oracle's
    backward-in-time solve (tuned and generic kernels)."""
    P = p + 1
    rng = np.random.default_rng(1400 + p + 3 * gamma)
    N, T, lam = 4096, 12.0, 0.8
    g = rng.standard_normal(N * P)
    zo, k, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-10, trans=True,
                                    opts=core.Opts(gamma=gamma))
    out = {}
    for on in (True, False):
        s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
        s.set_schedule(128, pairs=P <= 6)
        s.set_dense_bottom(on)
        z, _, _, cyc, _, st = s.adjoint_solve(dev(g), rtol=1e-10, max_cycles=80)
        out[on] = host(z)
        s.close()
        assert st == 0 and cyc[0] == k, (on, cyc, k)
        assert relerr(out[on], zo) <= TOL, (on, relerr(out[on], zo))
