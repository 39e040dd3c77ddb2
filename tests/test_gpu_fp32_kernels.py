"""GPU: each reduced-precision kernel of the FP32-inner defect correction
against the FP64 oracle on identical inputs (FP32-representable data, so the
only differences are the kernels' FP32 rounding and the FP32 rounding of the
tables).

Stated bounds, relative to the max-norm of the FP64 result, with
u = 2^-24 (FP32 unit roundoff) and P = p + 1 coefficients per slab:

* down leg (nu FP32 sweeps, residual in FP64 arithmetic, FP32 restriction):
  the iterate within c_S (nu + 1) P u, the restricted residual within
  c_R (nu + 1) P u of the larger of its own max-norm and the right-hand
  side's (the residual r = f - L u is a difference of terms of the size of
  f: where the sweeps nearly solve the slabs, large z, r is orders of
  magnitude below f, and the FP32 storage of u alone leaves an error of
  about u |f| in it, however exact the arithmetic);
* up leg (FP32 prolongation + correction, nu FP32 sweeps): within
  c_S (nu + 2) P u;
* the level-0 pass of an outer iteration (k_mix): the FP64 update of the
  iterate (u_out - u_in against the exact correction) within
  c_S (nu1 + nu2 + 2) P u, and the next inner restricted residual, on the
  pass's own u_out (identical inputs: the FP32 error of the update, times
  the norm of L, would otherwise reach it through f - L u_out), within
  c_R (nu1 + nu2 + nu1 + 3) P u of the larger of its own max-norm and that
  of the inner right-hand side f - L u_out (as for the down leg).

Each FP32 sweep evaluates P-term dot products (G f, c^T u) and a three-term
update, each with a rounding error of at most P u (resp. 3 u) of the
magnitudes involved, and the block Jacobi iteration does not amplify the
errors it carries by more than a small factor over a few sweeps; the
constants c_S and c_R absorb that factor and the ratio of the magnitudes
involved to the result's max-norm.  Their values are set from the measured
worst cases over p = 0..5, z = 1e-3 .. 4e3 (the test prints the measured
multiples).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
U32 = 2.0 ** -24
# measured worst multiples over the cases below: 0.72 (down-leg iterate),
# 0.44 (up leg), 0.32 (k_mix update) of the iterate unit; 1.03 (down-leg
# restricted residual) of the residual unit
C_S = 2.0
C_R = 4.0


def B():
    from paper_1409_5254_amd import binding
    return binding


def f32(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device=DEV)


def d64(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rep32(rng, n):
    """Random values that FP32 represents exactly."""
    return rng.standard_normal(n).astype(np.float32).astype(np.float64)


ZS = [1e-3, 1.0, 40.0, 4e3]


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("z", ZS)
@pytest.mark.parametrize("nsweep", [1, 2, 3])
def test_fp32_down_leg(p, z, nsweep):
    rng = np.random.default_rng(1000 + 10 * p + nsweep)
    N, P = 4096, p + 1
    s = B().Solver([N], [z * N], [1.0], p=p, precision=1)
    f, u = rep32(rng, N * P), rep32(rng, N * P)
    ref_u = core.sweeps(p, z, 1.0, f, u, nsweep)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, f, ref_u))
    out = torch.empty(N * P, dtype=torch.float32, device=DEV)
    rc = torch.empty(N // 2 * P, dtype=torch.float32, device=DEV)
    s.down32(0, f32(f), f32(u), out, rc, nsweep=nsweep)
    eu = relerr(host(out), ref_u)
    er = float(np.max(np.abs(host(rc) - ref_rc)) / max(np.max(np.abs(ref_rc)), np.max(np.abs(f))))
    unit = (nsweep + 1) * P * U32
    print(f"down32 p={p} z={z:g} nu={nsweep}: iterate {eu / unit:.3f}, rc {er / unit:.3f} "
          "x (nu+1) P u")
    assert eu <= C_S * unit
    assert er <= C_R * unit


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("z", ZS)
@pytest.mark.parametrize("nsweep", [0, 2, 3])
def test_fp32_up_leg(p, z, nsweep):
    rng = np.random.default_rng(2000 + 10 * p + nsweep)
    N, P = 4096, p + 1
    s = B().Solver([N], [z * N], [1.0], p=p, precision=1)
    f, u, e = rep32(rng, N * P), rep32(rng, N * P), rep32(rng, N // 2 * P)
    ref = core.sweeps(p, z, 1.0, f, core.prolong_add(p, e, u), nsweep)
    out = torch.empty(N * P, dtype=torch.float32, device=DEV)
    s.up32(0, f32(f), f32(u), f32(e), out, nsweep=nsweep)
    eu = relerr(host(out), ref)
    unit = (nsweep + 2) * P * U32
    print(f"up32 p={p} z={z:g} nu={nsweep}: {eu / unit:.3f} x (nu+2) P u")
    assert eu <= C_S * unit


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("z", ZS)
def test_mix_pass(p, z):
    """k_mix, one-level form: FP64 residual -> FP32 inner up leg -> FP64
    update -> FP32 next inner down leg, against the same steps in FP64."""
    rng = np.random.default_rng(3000 + p)
    N, P, u0 = 4096, p + 1, 0.75
    nu1, nu2 = 2, 2
    s = B().Solver([N], [z * N], [1.0], p=p, precision=1)
    f = rng.standard_normal(N * P)
    u = rng.standard_normal(N * P)
    e = rep32(rng, N // 2 * P) * 1e-2
    ff = core.fold(p, u0, f)
    r = core.residual(p, z, 1.0, ff, u)
    x = core.sweeps(p, z, 1.0, r, np.zeros_like(r), nu1)
    x = core.sweeps(p, z, 1.0, r, core.prolong_add(p, e, x), nu2)
    uo = torch.empty(N * P, dtype=torch.float64, device=DEV)
    rc = torch.empty(N // 2 * P, dtype=torch.float32, device=DEV)
    s.mix(d64(f), d64(u), f32(e), uo, rc, fold_u0=d64([u0]))
    un = host(uo)
    ex = relerr(un - u, x)
    # the next inner down leg from the pass's own u_out
    r2 = core.residual(p, z, 1.0, ff, un)
    y = core.sweeps(p, z, 1.0, r2, np.zeros_like(r2), nu1)
    ref_rc = core.restrict(p, core.residual(p, z, 1.0, r2, y))
    er = float(np.max(np.abs(host(rc) - ref_rc)) / max(np.max(np.abs(ref_rc)), np.max(np.abs(r2))))
    ux = (nu1 + nu2 + 2) * P * U32
    ur = (2 * nu1 + nu2 + 3) * P * U32
    print(f"mix p={p} z={z:g}: update {ex / ux:.3f} x (nu1+nu2+2) P u, "
          f"rc {er / ur:.3f} x (2nu1+nu2+3) P u")
    assert ex <= C_S * ux
    assert er <= C_R * ur


def test_fp32_ops_need_mixed_handle():
    s = B().Solver([256], [1.0], [1.0], p=1)
    x = torch.zeros(512, dtype=torch.float32, device=DEV)
    with pytest.raises(B().TmgError) as err:
        s.down32(0, x, x, x, None, nsweep=1)
    assert err.value.code == -9
