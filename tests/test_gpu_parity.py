"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative, max-norm over an instance):
* FP64 kernels and k cycles from identical inputs: 1e-12 -- the oracle and
  the kernels evaluate the same formulas in a different association order
  (the kernels use the rewritten sweep (1 - w) u + w A^{-1} f + w A^{-1} v w_left
  and fused multiply-adds), so the differences are a few ulp times the
  conditioning of at most a few dozen chained steps;
* converged solutions against the oracle's multigrid solve with the same
  number of cycles: 1e-12;
* converged solutions against the direct (sequential) solve: bounded by the
  residual tolerance, checked at 1e-8.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402
from workloads import gen  # noqa: E402

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
    """Error of a computed (restricted) residual, relative to the larger of
    its own max-norm and the right-hand side's: r = f - L u is a difference
    of terms of the size of f, and where the sweeps nearly solve the slabs
    (z of 1e3 and more) r is orders of magnitude below them, so that any
    rounding in the terms stands out against r alone."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), np.max(np.abs(rhs)), 1e-300))


def rand(rng, n):
    return rng.standard_normal(n)


# ---------------------------------------------------------------------------
# single kernels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("z", [1e-3, 1.0, 40.0, 1e3, 4e3])
@pytest.mark.parametrize("nsweep", [0, 1, 2, 3])
def test_down_kernel(p, z, nsweep):
    """k_down: nsweep damped block Jacobi sweeps (eq. chap4_ODESmoother), the
    residual and its restriction, with u0 folded, across several tiles and a
    ragged last tile."""
    rng = np.random.default_rng(p * 100 + nsweep)
    N = 4096
    T = z * N
    s = B().Solver([N], [T], [1.0], p=p)
    P = p + 1
    f, u = rand(rng, N * P), rand(rng, N * P)
    u0 = 0.7
    ff = core.fold(p, u0, f)
    ref_u = core.sweeps(p, z, 1.0, ff, u, nsweep)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, ff, ref_u))
    d_out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    d_rc = torch.empty(N // 2 * P, dtype=torch.float64, device=DEV)
    s.down(0, dev(f), dev(u), d_out, d_rc, nsweep=nsweep, fold_u0=dev([u0]))
    assert relerr(host(d_out), ref_u) <= TOL
    assert relerr_residual(host(d_rc), ref_rc, ff) <= TOL
    # zero initial guess
    ref0 = core.sweeps(p, z, 1.0, ff, np.zeros(N * P), nsweep)
    s.down(0, dev(f), None, d_out, None, nsweep=nsweep, fold_u0=dev([u0]))
    if nsweep:
        assert relerr(host(d_out), ref0) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("nsweep", [0, 2, 5])
@pytest.mark.parametrize("z", [0.3, 1e3, 4e3])
def test_up_kernel(p, nsweep, z):
    """k_up: prolongation + correction (eq. chap4_prolongationTime) then sweeps;
    z up to the stiffest slabs of the eigenmode batch (alpha ~ -2/z, omega = 1)."""
    rng = np.random.default_rng(7 + p)
    N = 2048
    s = B().Solver([N], [z * N], [1.0], p=p)
    P = p + 1
    f, u, e = rand(rng, N * P), rand(rng, N * P), rand(rng, N // 2 * P)
    ref = core.sweeps(p, z, 1.0, f, core.prolong_add(p, e, u), nsweep)
    out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    s.up(0, dev(f), dev(u), dev(e), out, nsweep=nsweep)
    assert relerr(host(out), ref) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("trans", [False, True])
def test_transposed_kernels(p, trans):
    """Transposed (adjoint) system, backward in time: sweeps with D^{-T},
    residual g - L^T z, same R and P."""
    rng = np.random.default_rng(11 + p)
    N, z = 1024, 0.05
    s = B().Solver([N], [z * N], [1.0], p=p)
    P = p + 1
    f, u, e = rand(rng, N * P), rand(rng, N * P), rand(rng, N // 2 * P)
    ref_u = core.sweeps(p, z, 1.0, f, u, 2, trans=trans)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, f, ref_u, trans=trans))
    d_out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    d_rc = torch.empty(N // 2 * P, dtype=torch.float64, device=DEV)
    s.down(0, dev(f), dev(u), d_out, d_rc, nsweep=2, trans=trans)
    assert relerr(host(d_out), ref_u) <= TOL
    assert relerr(host(d_rc), ref_rc) <= TOL
    ref_up = core.sweeps(p, z, 1.0, f, core.prolong_add(p, e, u), 2, trans=trans)
    s.up(0, dev(f), dev(u), dev(e), d_out, nsweep=2, trans=trans)
    assert relerr(host(d_out), ref_up) <= TOL
    norms = s.residual_norm(dev(f), dev(u), trans=trans)
    assert norms[0] == pytest.approx(np.linalg.norm(core.residual(p, z, 1.0, f, u, trans=trans)),
                                     rel=1e-12)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("N", [1, 2, 7, 256, 257, 1000, 4096])
@pytest.mark.parametrize("trans", [False, True])
def test_coarse_scan(p, N, trans):
    """k_coarse: the exact solve as an affine prefix scan equals sequential
    forward (backward) substitution."""
    rng = np.random.default_rng(N + p)
    for z in (1e-4, 2.0, 3e3):
        s = B().Solver([N], [z * N], [1.0], p=p, n_coarse=N)
        r = rand(rng, N * (p + 1))
        e = torch.empty(N * (p + 1), dtype=torch.float64, device=DEV)
        s.coarse_solve(0, dev(r), e, trans=trans)
        assert relerr(host(e), core.direct(p, z, 1.0, r, trans=trans)) <= 1e-12


@pytest.mark.parametrize("p", [0, 3])
def test_unit_damping_nilpotent(p):
    """Race guard: with omega = 1, N Jacobi sweeps from any start are the
    exact solve (the iteration matrix is nilpotent); a sweep that read an
    already-updated neighbour would still converge but break the count."""
    rng = np.random.default_rng(3)
    N, z = 16, 0.4
    s = B().Solver([N], [z * N], [1.0], p=p, omega_mode=1, omega=1.0, n_coarse=N)
    P = p + 1
    f, u = rand(rng, N * P), rand(rng, N * P)
    a, b = dev(u), torch.empty(N * P, dtype=torch.float64, device=DEV)
    for _ in range(N // 2):
        s.down(0, dev(f), a, b, None, nsweep=2)
        a, b = b, a
    assert relerr(host(a), core.direct(p, z, 1.0, f)) <= 1e-12


# ---------------------------------------------------------------------------
# cycles and solves
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("schedule", [-1, 0, 5])
def test_cycles_match_oracle(p, gamma, schedule):
    """k consecutive cycles from a random start (tmg_vcycle) equal the
    oracle's reference cycles (eq. chap4_errorTwoGridCycle applied
    recursively, V or W), whatever the split between the streaming kernels
    and the single-work-group bottom kernel (schedule = log2 of the largest
    level run inside one work-group; 0: only the coarsest solve there)."""
    rng = np.random.default_rng(40 + p)
    N, T, lam, u0 = 4096, 10.0, 1.3, 0.5
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma, schedule=schedule)
    P = p + 1
    f, u = rand(rng, N * P), rand(rng, N * P)
    du = dev(u)
    for _ in range(3):
        s.vcycle(dev(f), dev([u0]), du)
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, core.Opts(gamma=gamma))
    assert relerr(host(du), ref) <= TOL


@pytest.mark.parametrize("p", [0, 1, 3, 5])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("z", [1e3, 4e3])
def test_cycles_stiff(p, gamma, z):
    """Cycles at the stiff end of the eigenmode batch: the fine-level slab
    step z = lambda tau of 1e3 and 4e3 (alpha about -2/z, so omega* = 1 on
    every level), three cycles from a random start against the oracle."""
    rng = np.random.default_rng(int(z) + p)
    N, lam, u0 = 4096, 1.0, 0.5
    T = z * N / lam
    s = B().Solver([N], [T], [lam], p=p, gamma=gamma)
    P = p + 1
    f, u = rand(rng, N * P), rand(rng, N * P)
    du = dev(u)
    for _ in range(3):
        s.vcycle(dev(f), dev([u0]), du)
    ref = core.cycles(p, T, lam, core.fold(p, u0, f), u, 3, core.Opts(gamma=gamma))
    assert relerr(host(du), ref) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("opts", [dict(), dict(nu1=1, nu2=1), dict(nu1=3, nu2=0),
                                  dict(n_coarse=8), dict(omega_mode=1, omega=0.5)])
def test_solve_matches_oracle(p, opts):
    """tmg_solve: same cycle count as the oracle's solve to 1e-10 and the same
    iterate; the direct solve within the residual bound."""
    rng = np.random.default_rng(50 + p)
    N, T, lam, u0 = 2048, 20.0, 0.8, 1.0
    f = rand(rng, N * (p + 1)) * 0.01
    s = B().Solver([N], [T], [lam], p=p, **opts)
    res = s.solve(dev(f), dev([u0]), rtol=1e-10)
    uo, k, rr, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(**opts))
    assert res.status == 0 and res.cycles[0] == k
    assert res.relres[0] <= 1e-10
    assert relerr(host(res.u), uo) <= TOL
    ud = core.direct_solve(p, T, lam, u0, f)
    assert relerr(host(res.u), ud) <= 1e-8


def test_fourier_small_end_to_end():
    """Config 1: u' + u = f on (0, 10], p = 1, N = 1024, V(2,2) to 1e-10."""
    inst = gen.fourier_small().instances[0]
    s = B().Solver([inst.N], [inst.T], [inst.lam], p=1)
    res = s.solve(dev(inst.f), dev([inst.u0]), rtol=1e-10)
    uo, k, rr, _ = core.solve(1, inst.T, inst.lam, inst.u0, inst.f)
    assert res.cycles[0] == k == 11
    assert relerr(host(res.u), uo) <= TOL


@pytest.mark.parametrize("schedule", [-1, 0, 3])
@pytest.mark.parametrize("gamma", [1, 2])
def test_batched_uneven(schedule, gamma):
    """Several instances of different length and lambda in one handle,
    including one with a single level (N = n_coarse: the cycle is the exact
    solve) and, with schedule 3, instances whose level 1 runs in the bottom
    kernel (N = 16) next to ones whose level-1 up leg runs inside the
    level-0 pass; each equals its own oracle solve."""
    rng = np.random.default_rng(5)
    p = 1
    Ns = [2, 64, 1024, 4096, 512, 2048, 16]
    lams = [3.0, 0.5, 1.0, 2000.0, 7.0, 1e-3, 0.3]
    Ts = [1.0, 2.0, 10.0, 1.0, 5.0, 100.0, 0.5]
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rand(rng, n * (p + 1)) * 0.1 for n in Ns]
    s = B().Solver(Ns, Ts, lams, p=p, schedule=schedule, gamma=gamma)
    res = s.solve(dev(np.concatenate(fs)), dev(u0), rtol=1e-10)
    U = host(res.u)
    for j, n in enumerate(Ns):
        uo, k, rr, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j], opts=core.Opts(gamma=gamma))
        assert res.cycles[j] == k
        assert relerr(U[s.offsets[j]:s.offsets[j + 1]], uo) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("trans", [False, True])
def test_bottom_wavefront_levels(p, gamma, trans):
    """The bottom kernel runs levels of at most 64 * S slabs (S slabs per
    thread) in its first wavefront alone.  Instances whose bottom visit
    starts just above, at and below that size, plus a tiny one, solved in one
    handle (forward, or the adjoint system backward in time), each equal the
    oracle's solve with the same cycle count."""
    S = {0: 8, 1: 4}.get(p, 2)
    wave = 64 * S
    Ns = [4 * wave, 2 * wave, wave, wave // 2, 4]
    P = p + 1
    rng = np.random.default_rng(70 + p)
    lams = rng.uniform(0.2, 5.0, len(Ns))
    Ts = [float(n) / 64.0 for n in Ns]
    gs = [rand(rng, n * P) * 0.1 for n in Ns]
    s = B().Solver(Ns, Ts, list(lams), p=p, gamma=gamma)
    g = dev(np.concatenate(gs))
    if trans:
        z, _, _, cyc, _, st = s.adjoint_solve(g, rtol=1e-10)
    else:
        res = s.solve(g, dev(np.zeros(len(Ns))), rtol=1e-10)
        z, cyc, st = res.u, res.cycles, res.status
    assert st == 0
    Z = host(z)
    for j, n in enumerate(Ns):
        zo, k, _, _ = core.solve_folded(p, Ts[j], lams[j], gs[j], rtol=1e-10, trans=trans,
                                        opts=core.Opts(gamma=gamma))
        assert cyc[j] == k
        assert relerr(Z[s.offsets[j]:s.offsets[j + 1]], zo) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("schedule", [-1, 4])
def test_adjoint_solve_and_gradients(p, schedule):
    """tmg_adjoint_solve equals the oracle's multigrid solve of L^T z = g and
    its gradients equal the oracle's (which are pinned to finite
    differences).  Schedule 4 (levels of more than 16 slabs stream) runs the
    backward two-level level-0 pass and the paired levels."""
    rng = np.random.default_rng(60 + p)
    N, T, lam, u0 = 4096, 16.0, 1.7, 0.9
    f = rand(rng, N * (p + 1)) * 0.1
    y = rng.standard_normal(N)
    s = B().Solver([N], [T], [lam], p=p, schedule=schedule)
    fw = s.solve(dev(f), dev([u0]), rtol=1e-12)
    u = host(fw.u)
    g, _ = core.adjoint_rhs(p, u, y)
    z, dl, du0, cyc, rr, st = s.adjoint_solve(dev(g), u=fw.u, rtol=1e-12)
    zo, k, _, _ = core.solve_folded(p, T, lam, g, rtol=1e-12, trans=True)
    assert st == 0 and cyc[0] == k
    assert relerr(host(z), zo) <= TOL
    # gradients of the GPU's z (which equals the oracle's to 1e-12 above):
    # dlambda is a sum of N P products in another order, so its bar is the
    # summation bound 1e-12 |dl| + 16 eps tau sum |z_n M u_n|; du0 = v^T z_1
    zh = host(z)
    dlo, du0o = core.gradients(p, T / N, lam, u, zh)
    w = np.tile(1.0 / (2.0 * np.arange(p + 1) + 1.0), N)
    bound = 1e-12 * abs(dlo) + 16 * np.finfo(float).eps * (T / N) * np.sum(np.abs(zh * u * w))
    assert abs(dl[0] - dlo) <= bound
    assert du0[0] == pytest.approx(du0o, rel=1e-12)


# ---------------------------------------------------------------------------
# edge cases and errors
# ---------------------------------------------------------------------------

def test_zero_rhs_gives_zero():
    s = B().Solver([256], [1.0], [1.0], p=2)
    f = torch.zeros(256 * 3, dtype=torch.float64, device=DEV)
    u = torch.full_like(f, 5.0)
    res = s.solve(f, dev([0.0]), u=u)
    assert res.status == 0 and res.cycles[0] == 0 and float(host(u).max()) == 0.0


def test_max_cycles_and_nonfinite():
    s = B().Solver([1024], [10.0], [1.0], p=1)
    f = dev(np.random.default_rng(0).standard_normal(2048))
    res = s.solve(f, dev([1.0]), rtol=1e-10, max_cycles=2)
    assert res.status == B().TMG_NOT_CONVERGED and res.cycles[0] == 2 and res.relres[0] > 1e-10
    fb = f.clone()
    fb[17] = float("nan")
    with pytest.raises(B().TmgError) as ei:
        s.solve(fb, dev([1.0]))
    assert ei.value.code == -7


def test_warm_start_resume():
    """Checkpoint / resume: 3 cycles, copy out, 5 more cycles on a new
    handle equal 8 straight cycles bitwise."""
    rng = np.random.default_rng(9)
    N, p = 2048, 2
    f = dev(rand(rng, N * 3))
    s1 = B().Solver([N], [5.0], [1.0], p=p)
    a = torch.zeros(N * 3, dtype=torch.float64, device=DEV)
    for _ in range(8):
        s1.vcycle(f, dev([1.0]), a)
    b = torch.zeros_like(a)
    for _ in range(3):
        s1.vcycle(f, dev([1.0]), b)
    saved = host(b).copy()
    s2 = B().Solver([N], [5.0], [1.0], p=p)
    c = dev(saved)
    for _ in range(5):
        s2.vcycle(f, dev([1.0]), c)
    assert np.array_equal(host(c), host(a))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("trans", [False, True])
def test_fused_level0_pass(p, trans):
    """tmg_op_fused: the pass every cycle after the first runs at level 0 --
    recomputed nu1 sweeps, correction, nu2 sweeps (u_out), then nu1 sweeps,
    residual and restriction (rc)."""
    rng = np.random.default_rng(70 + p)
    N, z = 4096, 0.02
    s = B().Solver([N], [z * N], [1.0], p=p)
    P = p + 1
    f, u, e = rand(rng, N * P), rand(rng, N * P), rand(rng, N // 2 * P)
    u0 = None if trans else 0.3
    ff = f if trans else core.fold(p, u0, f)
    post = core.sweeps(p, z, 1.0, ff, core.prolong_add(p, e, core.sweeps(p, z, 1.0, ff, u, 2,
                                                                         trans=trans)), 2,
                       trans=trans)
    nxt = core.sweeps(p, z, 1.0, ff, post, 2, trans=trans)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, ff, nxt, trans=trans))
    d_out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    d_rc = torch.empty(N // 2 * P, dtype=torch.float64, device=DEV)
    s.fused(dev(f), dev(u), dev(e), d_out, d_rc, trans=trans,
            fold_u0=None if trans else dev([u0]))
    assert relerr(host(d_out), post) <= TOL
    assert relerr(host(d_rc), ref_rc) <= TOL


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("trans", [False, True])
def test_fused2_level0_pass(p, trans):
    """tmg_op_fused2: level 1's correction computed in the tiles as level
    1's first-visit up leg (nu1 sweeps from zero on f1, correction with the
    level-2 e2, nu2 sweeps at tau_1 = 2 tau), then the pass of tmg_op_fused,
    then level 1's next down leg into f2."""
    rng = np.random.default_rng(80 + p)
    N, z = 4096, 0.02
    s = B().Solver([N], [z * N], [1.0], p=p)
    P = p + 1
    f, u = rand(rng, N * P), rand(rng, N * P)
    f1, e2 = rand(rng, N // 2 * P), rand(rng, N // 4 * P)
    u0 = None if trans else 0.3
    ff = f if trans else core.fold(p, u0, f)
    e1 = core.sweeps(p, 2 * z, 1.0, f1, np.zeros(N // 2 * P), 2, trans=trans)
    e1 = core.sweeps(p, 2 * z, 1.0, f1, core.prolong_add(p, e2, e1), 2, trans=trans)
    post = core.sweeps(p, z, 1.0, ff, core.prolong_add(p, e1, core.sweeps(p, z, 1.0, ff, u, 2,
                                                                          trans=trans)), 2,
                       trans=trans)
    nxt = core.sweeps(p, z, 1.0, ff, post, 2, trans=trans)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, ff, nxt, trans=trans))
    # level 1's next down leg on rc (tau_1 = 2 tau): sweeps from zero,
    # residual, restriction
    x1 = core.sweeps(p, 2 * z, 1.0, ref_rc, np.zeros(N // 2 * P), 2, trans=trans)
    ref_f2 = core.restrict(p, core.residual(p, 2 * z, 1.0, ref_rc, x1, trans=trans))
    d_out = torch.empty(N * P, dtype=torch.float64, device=DEV)
    d_rc = torch.empty(N // 2 * P, dtype=torch.float64, device=DEV)
    d_f2 = torch.empty(N // 4 * P, dtype=torch.float64, device=DEV)
    s.fused2(dev(f), dev(u), dev(f1), dev(e2), d_out, d_rc, f2=d_f2, trans=trans,
             fold_u0=None if trans else dev([u0]))
    assert relerr(host(d_out), post) <= TOL
    assert relerr(host(d_rc), ref_rc) <= TOL
    assert relerr(host(d_f2), ref_f2) <= TOL


def test_many_array_sets_on_one_handle():
    """Solves on more distinct (f, u) arrays than the handle keeps graphs
    for: each solve still equals the oracle (the graph cache is emptied only
    between solves, never between the graphs one solve launches)."""
    rng = np.random.default_rng(11)
    p, N, T, lam = 1, 512, 3.0, 0.7
    s = B().Solver([N], [T], [lam], p=p)
    for i in range(9):
        f = rand(rng, N * (p + 1)) * 0.1
        res = s.solve(dev(f), dev([0.5]), rtol=1e-10)
        uo, k, _, _ = core.solve(p, T, lam, 0.5, f)
        assert res.status == 0 and res.cycles[0] == k
        assert relerr(host(res.u), uo) <= TOL
