"""GPU: FP32-inner / FP64-outer defect correction (precision = 1).

Each outer iteration computes r = f - L u in FP64, runs one cycle on
L e = r with FP32 storage and FP32 smoothing / restriction / prolongation
(intra-cycle residuals in FP64 arithmetic, coarsest levels in FP64) and
updates u += e in FP64.  The FP32 rounding differs from the oracle's FP32
reference (different operation order), so parity is stated as:
* the outer iteration count within 1 of the oracle's mixed solve and of the
  FP64 solve;
* the converged solution within 1e-8 (relative, max-norm) of the direct
  solve, the same bound as the FP64 solve (the residual tolerance decides);
* one mixed iteration against one FP64 cycle from the same iterate: the
  corrections agree to 1e-5 relative (FP32 unit roundoff ~6e-8 times the
  conditioning of a few dozen chained FP32 steps).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402
from workloads import gen  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def B():
    from paper_1409_5254_amd import binding
    return binding


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("schedule", [-1, 0])
@pytest.mark.parametrize("gamma", [1, 2])
def test_mixed_solve(p, schedule, gamma):
    w = gen.long_horizon(B=1, N=1 << 12, T=1e4 * 2 ** -12)
    inst = w.instances[0]
    r = np.random.default_rng(5)
    f = gen.fourier_load(p, inst.N, inst.T, r.standard_normal(16), r.uniform(0, 2 * np.pi, 16))
    s = B().Solver([inst.N], [inst.T], [inst.lam], p=p, precision=1, schedule=schedule,
                   gamma=gamma)
    res = s.solve(dev(f), dev([inst.u0]), rtol=1e-10)
    opts = core.Opts(gamma=gamma)
    _, km, _, _ = core.solve_mixed(p, inst.T, inst.lam, inst.u0, f, opts=opts)
    _, k64, _, _ = core.solve(p, inst.T, inst.lam, inst.u0, f, opts=opts)
    assert res.status == 0 and res.relres[0] <= 1e-10
    assert abs(res.cycles[0] - km) <= 1 and abs(res.cycles[0] - k64) <= 1
    ud = core.direct_solve(p, inst.T, inst.lam, inst.u0, f)
    assert relerr(host(res.u), ud) <= 1e-8


@pytest.mark.parametrize("p", [1, 3])
def test_mixed_iteration_against_fp64_cycle(p):
    """One defect-correction step (tmg_vcycle with precision = 1) against one
    FP64 cycle from the same iterate: the corrections agree to 1e-5."""
    rng = np.random.default_rng(9)
    N, T, lam = 4096, 50.0, 2.0
    f = rng.standard_normal(N * (p + 1)) * 0.01
    u = rng.standard_normal(N * (p + 1)) * 0.01
    s64 = B().Solver([N], [T], [lam], p=p, schedule=0)
    s32 = B().Solver([N], [T], [lam], p=p, schedule=0, precision=1)
    a, b = dev(u), dev(u)
    s64.vcycle(dev(f), dev([0.5]), a)
    s32.vcycle(dev(f), dev([0.5]), b)
    da, db = host(a) - u, host(b) - u
    err = relerr(db, da)
    assert err <= 1e-5
    ref = core.cycles(p, T, lam, core.fold(p, 0.5, f), u, 1)
    assert relerr(host(a), ref) <= 1e-12


def test_mixed_batched_and_adjoint():
    """Uneven batch in mixed precision; the adjoint solve in mixed precision
    matches the FP64 adjoint to the residual bound."""
    rng = np.random.default_rng(11)
    p = 1
    Ns = [1 << 12, 1 << 14, 1 << 11, 2]
    lams = [1.0, 30.0, 0.2, 5.0]
    Ts = [10.0, 5.0, 100.0, 1.0]
    fs = [rng.standard_normal(n * 2) * 0.1 for n in Ns]
    u0 = rng.uniform(-1, 1, len(Ns))
    s = B().Solver(Ns, Ts, lams, p=p, precision=1)
    res = s.solve(dev(np.concatenate(fs)), dev(u0), rtol=1e-10)
    U = host(res.u)
    for j in range(len(Ns)):
        ud = core.direct_solve(p, Ts[j], lams[j], u0[j], fs[j])
        assert relerr(U[s.offsets[j]:s.offsets[j + 1]], ud) <= 1e-8
    g = np.concatenate([rng.standard_normal(n * 2) for n in Ns])
    z, dl, du, cyc, rr, st = s.adjoint_solve(dev(g), u=res.u, rtol=1e-10)
    Z = host(z)
    assert st == 0
    for j in range(len(Ns)):
        zd = core.direct(p, Ts[j] / Ns[j], lams[j], g[s.offsets[j]:s.offsets[j + 1]], trans=True)
        assert relerr(Z[s.offsets[j]:s.offsets[j + 1]], zd) <= 1e-8
