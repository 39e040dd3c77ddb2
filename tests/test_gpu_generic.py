"""GPU parity of the generic kernels against the FP64 oracle: degrees above
the tuned kernels' (p = 6 .. 20, the paper's p = 10 and 20 included) and the
time-periodic problem u(0) = u(T) (section 3, eqs.
chap4_equationLinearSystemODEPeriodic, chap4_circulantMatrix) at every
degree.

Bars as for the tuned kernels: 1e-12 relative (max-norm per instance) for
kernels, cycles and same-count solves; a restricted residual against the
larger of its max-norm and the right-hand side's; 1e-8 against the direct
(or periodic direct) solve; the two-grid contraction between 0.9 and
1 + 1e-5 times the Fourier estimate, which is exact for periodic problems.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import analysis as an  # noqa: E402
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


def relerr_residual(a, b, rhs):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), np.max(np.abs(rhs)), 1e-300))


# (p, periodic) cases: the high degrees, and the periodic problem
HIGH = [6, 10, 15, 20]
PER = [0, 1, 3, 5, 10]


@pytest.mark.parametrize("p,periodic", [(p, False) for p in HIGH] + [(p, True) for p in PER])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("z", [1e-3, 1.0, 40.0])
def test_generic_legs(p, periodic, trans, z):
    """Down leg (sweeps, residual, restriction; u0 folded for the forward
    initial-value problem) and up leg (prolongation, sweeps), over several
    tiles and a ragged last one."""
    rng = np.random.default_rng(500 + p + (7 if periodic else 0))
    N = 1024
    P = p + 1
    s = B().Solver([N], [z * N], [1.0], p=p, periodic=int(periodic))
    f, u, e = (rng.standard_normal(n) for n in (N * P, N * P, N // 2 * P))
    u0 = 0.0 if (periodic or trans) else 0.7
    ff = core.fold(p, u0, f)
    kw = dict(trans=trans, periodic=periodic)
    ref_u = core.sweeps(p, z, 1.0, ff, u, 2, **kw)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, ff, ref_u, **kw))
    out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    rc = torch.empty(N // 2 * P, dtype=torch.float64, device=DEV)
    fold = None if (periodic or trans) else dev([u0])
    s.down(0, dev(f), dev(u), out, rc, nsweep=2, trans=trans, fold_u0=fold)
    assert relerr(host(out), ref_u) <= TOL
    assert relerr_residual(host(rc), ref_rc, ff) <= TOL
    ref_up = core.sweeps(p, z, 1.0, ff, core.prolong_add(p, e, u), 3, **kw)
    s.up(0, dev(f), dev(u), dev(e), out, nsweep=3, trans=trans, fold_u0=fold)
    assert relerr(host(out), ref_up) <= TOL
    norms = s.residual_norm(dev(f), dev(u), trans=trans, fold_u0=fold)
    assert norms[0] == pytest.approx(np.linalg.norm(core.residual(p, z, 1.0, ff, u, **kw)),
                                     rel=1e-12)
    s.close()


@pytest.mark.parametrize("p", [0, 2, 5, 10, 20])
@pytest.mark.parametrize("N", [1, 2, 7, 256, 1000, 4096])
@pytest.mark.parametrize("trans", [False, True])
def test_periodic_exact_solve(p, N, trans):
    """The coarsest-level solve of the periodic system: the affine prefix
    scan closed cyclically equals the oracle's periodic direct solve.  Two
    things of the problem itself scale the bar: the closure divides by
    1 - alpha^N (alpha^N ~ exp(-lambda T)), up to 1 / (lambda T) for a short
    horizon; and the end values are sums over N_eff = min(N, 1 / (1 - |alpha|))
    slabs (alpha ~ 1 - z for small z), whose rounding grows with N_eff (the
    oracle's sequential substitution and the GPU's scan add them in different
    orders).  Bar: 1e-12 max(1, N_eff / 1000) max(1, 1 / |1 - alpha^N|)."""
    rng = np.random.default_rng(N + 31 * p)
    for z in (1e-4, 2.0, 3e3):
        s = B().Solver([N], [z * N], [1.0], p=p, n_coarse=N, periodic=1)
        r = rng.standard_normal(N * (p + 1))
        e = torch.empty(N * (p + 1), dtype=torch.float64, device=DEV)
        s.coarse_solve(0, dev(r), e, trans=trans)
        ref = core.direct(p, z, 1.0, r, trans=trans, periodic=True)
        al = an.alpha_of(p, z)
        cond = 1.0 / abs(1.0 - al ** N)
        neff = min(N, 1.0 / max(1.0 - abs(al), 1e-300))
        bar = TOL * max(1.0, neff / 1000.0) * max(1.0, cond)
        assert relerr(host(e), ref) <= bar, (z, cond, neff)
        s.close()


@pytest.mark.parametrize("p,periodic", [(6, False), (10, False), (20, False), (0, True),
                                        (1, True), (3, True), (5, True), (10, True)])
@pytest.mark.parametrize("gamma", [1, 2])
def test_generic_cycles(p, periodic, gamma):
    """Three cycles from a random start (tmg_vcycle) equal the oracle's."""
    rng = np.random.default_rng(600 + p)
    N, T, lam, u0 = 2048, 12.0, 1.3, 0.5
    P = p + 1
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma, periodic=int(periodic))
    f, u = rng.standard_normal(N * P), rng.standard_normal(N * P)
    du = dev(u)
    for _ in range(3):
        s.vcycle(dev(f), dev([u0]), du)
    ff = f if periodic else core.fold(p, u0, f)
    ref = core.cycles(p, T, lam, ff, u, 3, core.Opts(gamma=gamma), periodic=periodic)
    assert relerr(host(du), ref) <= TOL
    s.close()


@pytest.mark.parametrize("p,periodic", [(10, False), (20, False), (6, False), (0, True),
                                        (2, True), (4, True), (10, True)])
@pytest.mark.parametrize("opts", [dict(), dict(nu1=1, nu2=1), dict(n_coarse=8, gamma=2),
                                  dict(omega_mode=1, omega=0.5)])
def test_generic_solve(p, periodic, opts):
    """tmg_solve: the oracle's cycle count and iterate, and the direct (or
    periodic direct) solve within the residual bound."""
    rng = np.random.default_rng(700 + p)
    N, T, lam, u0 = 4096, 20.0, 0.8, 1.0
    P = p + 1
    f = rng.standard_normal(N * P) * 0.01
    s = B().Solver([N], [T], [lam], p=p, periodic=int(periodic), **opts)
    res = s.solve(dev(f), dev([u0]), rtol=1e-10)
    ff = f if periodic else core.fold(p, u0, f)
    uo, k, _, _ = core.solve_folded(p, T, lam, ff, opts=core.Opts(**opts), periodic=periodic)
    assert res.status == 0 and res.cycles[0] == k, (res.cycles, k)
    assert relerr(host(res.u), uo) <= TOL
    ud = core.direct(p, T / N, lam, ff, periodic=periodic)
    assert relerr(host(res.u), ud) <= 1e-8
    s.close()


@pytest.mark.parametrize("p,periodic", [(10, False), (3, True)])
def test_generic_adjoint_and_gradients(p, periodic):
    """The adjoint solve (L^T z = g backward in time) equals the oracle's;
    the gradient dlambda within the summation bound of the oracle's value
    from the GPU's z."""
    rng = np.random.default_rng(800 + p)
    N, T, lam = 2048, 16.0, 1.7
    P = p + 1
    f = rng.standard_normal(N * P) * 0.1
    y = rng.standard_normal(N)
    s = B().Solver([N], [T], [lam], p=p, periodic=int(periodic))
    fw = s.solve(dev(f), dev([0.9]), rtol=1e-12)
    u = host(fw.u)
    g, _ = core.adjoint_rhs(p, u, y)
    z, dl, du0, cyc, rr, st = s.adjoint_solve(dev(g), u=fw.u, rtol=1e-12)
    zo, k, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-12, trans=True, periodic=periodic)
    assert st == 0 and cyc[0] == k
    assert relerr(host(z), zo) <= TOL
    zh = host(z)
    dlo, _ = core.gradients(p, T / N, lam, u, zh)
    w = np.tile(1.0 / (2.0 * np.arange(P) + 1.0), N)
    bound = 1e-12 * abs(dlo) + 16 * np.finfo(float).eps * (T / N) * np.sum(np.abs(zh * u * w))
    assert abs(dl[0] - dlo) <= bound
    s.close()


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("gamma", [1, 2])
def test_generic_batched_uneven(periodic, gamma):
    """Instances of different length and lambda in one handle, one of them a
    single level (N = n_coarse: the cycle is the exact solve)."""
    rng = np.random.default_rng(900)
    p = 10 if not periodic else 2
    Ns = [2, 64, 1024, 4096, 512]
    lams = [3.0, 0.5, 1.0, 2000.0, 7.0]
    Ts = [1.0, 2.0, 10.0, 1.0, 5.0]
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rng.standard_normal(n * (p + 1)) * 0.1 for n in Ns]
    s = B().Solver(Ns, Ts, lams, p=p, gamma=gamma, periodic=int(periodic))
    res = s.solve(dev(np.concatenate(fs)), dev(u0), rtol=1e-10)
    U = host(res.u)
    for j, n in enumerate(Ns):
        ff = fs[j] if periodic else core.fold(p, u0[j], fs[j])
        uo, k, _, _ = core.solve_folded(p, Ts[j], lams[j], ff, opts=core.Opts(gamma=gamma),
                                        periodic=periodic)
        assert res.cycles[j] == k, (j, res.cycles[j], k)
        assert relerr(U[s.offsets[j]:s.offsets[j + 1]], uo) <= TOL
    s.close()


@pytest.mark.parametrize("p,z,nu", [(0, 1e-3, 1), (1, 1e-3, 1), (1, 1.0, 2), (3, 0.1, 1),
                                    (5, 1e-2, 1), (2, 10.0, 5)])
def test_periodic_two_grid_contraction(p, z, nu):
    """The two-grid cycle (coarse level N/2 solved exactly, cyclically) on the
    periodic problem, N = 1024, f = 0, random start: first cycles equal the
    oracle's, and the measured contraction lies under the Fourier estimate
    (exact for periodic problems) and above 0.9 of it."""
    N = 1024
    P = p + 1
    rng = np.random.default_rng(200 + p)
    start = rng.uniform(0.0, 1.0, N * P)
    s = B().Solver([N], [z * N], [1.0], p=p, nu1=nu, nu2=nu, n_coarse=N // 2, periodic=1)
    f = torch.zeros(N * P, dtype=torch.float64, device=DEV)
    u0 = torch.zeros(1, dtype=torch.float64, device=DEV)
    u = dev(start)
    r = [float(s.residual_norm(f, u)[0])]
    opts = core.Opts(nu1=nu, nu2=nu, gamma=1, n_coarse=N // 2)
    uo = start.copy()
    while len(r) < 40 and r[-1] > 1e-200 * r[0]:
        s.vcycle(f, u0, u)
        r.append(float(s.residual_norm(f, u)[0]))
        if len(r) <= 4:
            uo = core.cycles(p, z * N, 1.0, np.zeros_like(uo), uo, 1, opts, periodic=True)
            assert np.max(np.abs(host(u) - uo)) <= 1e-12 * np.max(np.abs(start))
    K = len(r) - 1
    est = an.two_grid_rho(p, z, nu, nu, N=N)
    if r[-1] > 1e-200 * r[0]:
        tail = (r[K] / r[K // 2]) ** (1.0 / (K - K // 2))
        assert 0.9 * est <= tail <= (1.0 + 1e-5) * est, (tail, est)
    else:
        assert est < 1e-4
    s.close()


@pytest.mark.parametrize("p", [6, 9, 10, 15, 20])
@pytest.mark.parametrize("gamma", [1, 2])
def test_generic_bottom_visit_bitwise(p, gamma):
    """The generic bottom visit (one work-group runs the levels up to the
    bottom cap, k_gvisit) computes each slab's steps as the one-level legs
    and the coarsest level's exact solve do: a solve and an adjoint solve
    give the same bits with the bottom cap at the coarsest level (every
    other level streams), at 8 and 32 slabs, and at the largest (256 slabs
    up to p = 9, 128 above); and they equal the oracle's at 1e-12."""
    rng = np.random.default_rng(1000 + p + 10 * gamma)
    N, T, lam, u0 = 2048, 8.0, 0.9, 0.6
    P = p + 1
    f = rng.standard_normal(N * P) * 0.1
    g = rng.standard_normal(N * P) * 0.1
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
    s.set_dense_bottom(False)   # the recursion at every visit (compared bit for bit)
    out = []
    largest = 256 if P <= 10 else 128
    for cap in (2, 8, 32, largest):
        s.set_schedule(cap, pairs=False)
        r = s.solve(dev(f), dev([u0]), rtol=1e-10)
        z, _, _, cz, _, st = s.adjoint_solve(dev(g), rtol=1e-10)
        assert r.status == 0 and st == 0
        out.append((host(r.u).copy(), list(r.cycles), host(z).copy(), list(cz)))
    s.close()
    for o in out[1:]:
        assert o[1] == out[0][1] and o[3] == out[0][3]
        assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[2], out[0][2])
    uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(gamma=gamma))
    assert out[0][1][0] == k
    assert relerr(out[0][0], uo) <= TOL
    zo, kz, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-10, trans=True,
                                     opts=core.Opts(gamma=gamma))
    assert out[0][3][0] == kz
    assert relerr(out[0][2], zo) <= TOL


def test_generic_schedule_caps():
    """A generic handle takes bottom caps from the coarsest level up to its
    bottom visit's largest level (the periodic problem's too), without
    two-level launches or spans."""
    s = B().Solver([1024], [1.0], [1.0], p=10)
    s.set_schedule(128, pairs=False)
    s.set_schedule(2, pairs=False)
    with pytest.raises(B().TmgError):
        s.set_schedule(256, pairs=False)
    with pytest.raises(B().TmgError):
        s.set_schedule(64, pairs=True)
    s.close()
    s = B().Solver([1024], [1.0], [1.0], p=3, periodic=1)
    s.set_schedule(2, pairs=False)
    s.set_schedule(256, pairs=False)
    with pytest.raises(B().TmgError):
        s.set_schedule(512, pairs=False)
    s.close()


@pytest.mark.parametrize("p", [6, 10, 15, 20])
@pytest.mark.parametrize("gamma", [1, 2])
def test_generic_dense_bottom(p, gamma):
    """One instance's bottom visits as the tabulated dense operator on the
    generic kernels (its columns are k_gvisit's visits of the unit loads):
    three cycles from a random start and a solve, at the largest bottom
    level (256 slabs up to p = 9, 128 above: 1408 to 2688 unknowns), against
    the oracle at 1e-12 with the same cycle count."""
    rng = np.random.default_rng(1100 + p + 10 * gamma)
    N, T, lam, u0 = 4096, 8.0, 1.1, 0.4
    P = p + 1
    f, u = rng.standard_normal(N * P) * 0.1, rng.standard_normal(N * P)
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
    s.set_schedule(256 if P <= 10 else 128, pairs=False)
    du = dev(u)
    for _ in range(3):
        s.vcycle(dev(f), dev([u0]), du)
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, core.Opts(gamma=gamma))
    assert relerr(host(du), ref) <= TOL
    res = s.solve(dev(f), dev([u0]), rtol=1e-10)
    uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(gamma=gamma))
    assert res.status == 0 and res.cycles[0] == k
    assert relerr(host(res.u), uo) <= TOL
    s.close()


@pytest.mark.parametrize("p", [0, 3, 10])
@pytest.mark.parametrize("gamma", [1, 2])
def test_periodic_bottom_visit(p, gamma):
    """The periodic problem's bottom visit (every level wraps around: slab
    -1 is slab N_l - 1; the coarsest level closes cyclically): solves and
    adjoint solves with bottom caps 2, 8, 32 and the largest give the same
    bits with the dense operator off, and equal the oracle's periodic
    solves at 1e-12; with the operator on (one instance), the same cycle
    count and 1e-12."""
    rng = np.random.default_rng(1600 + p + 10 * gamma)
    N, T, lam = 2048, 8.0, 0.9
    P = p + 1
    f = rng.standard_normal(N * P) * 0.1
    g = rng.standard_normal(N * P) * 0.1
    largest = 256 if P <= 10 else 128
    uo, k, _, _ = core.solve_folded(p, T, lam, f, opts=core.Opts(gamma=gamma), periodic=True)
    zo, kz, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-10, trans=True,
                                     opts=core.Opts(gamma=gamma), periodic=True)
    for dense in (False, True):
        s = B().Solver([N], [T], [lam], p=p, gamma=gamma, periodic=1)
        s.set_dense_bottom(dense)
        out = []
        for cap in ((2, 8, 32, largest) if not dense else (largest,)):
            s.set_schedule(cap, pairs=False)
            r = s.solve(dev(f), dev([0.0]), rtol=1e-10)
            z, _, _, cz, _, st = s.adjoint_solve(dev(g), rtol=1e-10)
            assert r.status == 0 and st == 0
            out.append((host(r.u).copy(), list(r.cycles), host(z).copy(), list(cz)))
        s.close()
        for o in out:
            assert o[1][0] == k and o[3][0] == kz, (dense, o[1], k, o[3], kz)
            assert relerr(o[0], uo) <= TOL and relerr(o[2], zo) <= TOL
        if not dense:
            for o in out[1:]:
                assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[2], out[0][2])
