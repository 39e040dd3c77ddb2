"""The schedule autotuner: whatever schedule it installs, solves still equal
the oracle (the schedule only moves work between kernels)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("gamma", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_then_solve(gamma, precision):
    from paper_1409_5254_amd import binding as B
    rng = np.random.default_rng(90 + gamma)
    p = 1
    Ns = [4096, 64, 16384, 256, 2]
    lams = [1.0, 7.0, 0.2, 30.0, 2.0]
    Ts = [10.0, 1.0, 50.0, 2.0, 1.0]
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rng.standard_normal(n * (p + 1)) * 0.1 for n in Ns]
    s = B.Solver(Ns, Ts, lams, p=p, gamma=gamma, precision=precision)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    before = s.solve(f, d0, rtol=1e-10)
    U0 = host(before.u).copy()
    cap, pairs, direct = s.autotune(f, d0, torch.empty_like(f))
    assert cap >= 2
    if gamma == 2:
        assert pairs  # two-level launches are a V-cycle schedule only
    after = s.solve(f, d0, rtol=1e-10)
    U1 = host(after.u)
    assert after.status == 0
    for j, n in enumerate(Ns):
        seg = slice(s.offsets[j], s.offsets[j + 1])
        if precision == 0:
            uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j], opts=core.Opts(gamma=gamma))
            assert after.cycles[j] == k == before.cycles[j]
            assert relerr(U1[seg], uo) <= 1e-12
        else:
            ud = core.direct_solve(p, Ts[j], lams[j], u0[j], fs[j])
            assert abs(after.cycles[j] - before.cycles[j]) <= 1
            assert relerr(U1[seg], ud) <= 1e-8
        assert relerr(U1[seg], U0[seg]) <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("cap", [32, 256])
def test_direct_launches_match_graphs(precision, cap):
    """Cycles launched kernel by kernel run the same kernels in the same
    order as the captured graphs: bitwise the same iterate and counts."""
    from paper_1409_5254_amd import binding as B
    rng = np.random.default_rng(7 + cap)
    p = 3
    Ns = [8192, 512, 32768]
    lams = [1.0, 4.0, 0.5]
    Ts = [40.0, 2.0, 100.0]
    u0 = rng.uniform(-1, 1, len(Ns))
    f = dev(np.concatenate([rng.standard_normal(n * (p + 1)) for n in Ns]))
    d0 = dev(u0)
    s = B.Solver(Ns, Ts, lams, p=p, precision=precision)
    out = {}
    for direct in (False, True, False):
        s.set_schedule(cap, pairs=True, direct=direct)
        r = s.solve(f, d0, rtol=1e-10)
        assert r.status == 0
        out.setdefault(direct, []).append((host(r.u).copy(), list(r.cycles)))
    for (ua, ca) in out[True] + out[False][1:]:
        ub, cb = out[False][0]
        assert ca == cb
        assert np.array_equal(ua, ub)
    if precision == 0:
        for j, n in enumerate(Ns):
            seg = slice(s.offsets[j], s.offsets[j + 1])
            fj = host(f)[seg]
            uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], fj, opts=core.Opts())
            assert out[True][0][1][j] == k
            assert relerr(out[True][0][0][seg], uo) <= 1e-12


def test_set_schedule_rejects_bad_cap():
    from paper_1409_5254_amd import binding as B
    s = B.Solver([1024], [1.0], [1.0], p=1)
    with pytest.raises(B.TmgError):
        s.set_schedule(1, pairs=True)
    with pytest.raises(B.TmgError):
        s.set_schedule(1 << 30, pairs=True)
