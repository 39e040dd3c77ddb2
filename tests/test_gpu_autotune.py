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
    sch = s.autotune(f, d0, torch.empty_like(f))
    assert sch["bottom_cap"] >= 2
    if gamma == 2:
        # two-level launches and spans are V-cycle schedules only
        assert sch["pairs"] and sch["span"] == 0
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


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("span", [3, 4])
@pytest.mark.parametrize("cap", [8, 64])
def test_span_schedule_matches_pairs(precision, span, cap):
    """Spans compute every step of the pair and single launches in the same
    order: the same iterate to the last bit, forward and adjoint, also for
    instances whose bottom level falls inside a span."""
    from paper_1409_5254_amd import binding as B
    rng = np.random.default_rng(11 * span + cap)
    p = 3
    # lb = log2(N / cap) levels stream: 3 .. 11, so spans end at and before
    # every instance's bottom level
    Ns = [cap << 3, cap << 5, cap << 7, cap << 11, cap << 6, 2]
    lams = [1.0, 4.0, 0.5, 2.0, 9.0, 1.0]
    Ts = [4.0, 20.0, 60.0, 900.0, 30.0, 1.0]
    u0 = rng.uniform(-1, 1, len(Ns))
    fh = np.concatenate([rng.standard_normal(n * (p + 1)) for n in Ns])
    f, d0 = dev(fh), dev(u0)
    s = B.Solver(Ns, Ts, lams, p=p, precision=precision)
    res = {}
    # span_after counts streaming levels below level 1 before the spans:
    # 1 (a lone level), 2 (a pair), 3 (a pair and a lone level)
    for sp, after in ((0, 2), (span, 1), (span, 2), (span, 3)):
        s.set_schedule(cap, pairs=True, span=sp, span_after=after)
        r = s.solve(f, d0, rtol=1e-10)
        assert r.status == 0
        u = host(r.u).copy()
        g = dev(u - 0.5)
        z, dl, du, cz, _, st = s.adjoint_solve(g, u=r.u)
        assert st == 0
        res[(sp, after)] = (u, list(r.cycles), host(z).copy(), cz, dl, du)
    a = res[(0, 2)]
    for key in ((span, 1), (span, 2), (span, 3)):
        b = res[key]
        assert a[1] == b[1] and a[3] == b[3]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
        assert a[4] == b[4] and a[5] == b[5]
    b = res[(span, 1)]
    if precision == 0:
        for j, n in enumerate(Ns):
            seg = slice(s.offsets[j], s.offsets[j + 1])
            uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], fh[seg])
            assert b[1][j] == k
            assert relerr(b[0][seg], uo) <= 1e-12


def test_span_schedule_rejected_where_it_cannot_run():
    from paper_1409_5254_amd import binding as B
    s = B.Solver([4096], [1.0], [1.0], p=1, gamma=2)
    with pytest.raises(B.TmgError):
        s.set_schedule(64, pairs=True, span=4)
    s = B.Solver([4096], [1.0], [1.0], p=1)
    with pytest.raises(B.TmgError):
        s.set_schedule(64, pairs=False, span=4)
    with pytest.raises(B.TmgError):
        s.set_schedule(64, pairs=True, span=5)
    with pytest.raises(B.TmgError):
        s.set_schedule(64, pairs=True, span=4, span_after=0)
    s.set_schedule(64, pairs=True, span=4, span_after=2)
