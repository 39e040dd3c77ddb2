"""The host side of a solve: it follows every instance's state through the
copy the device writes into pinned host memory after each cycle, queues
cycles ahead, and stops when every instance has finished.  Whatever it
queues, the iterate, the cycle counts and the relative residuals must be
those of the oracle's solve with the same tolerance and cycle cap."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402

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


def _case(seed, Ns, p):
    rng = np.random.default_rng(seed)
    lams = list(rng.uniform(0.5, 20.0, len(Ns)))
    Ts = list(rng.uniform(1.0, 40.0, len(Ns)))
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rng.standard_normal(n * (p + 1)) for n in Ns]
    return lams, Ts, u0, fs


@pytest.mark.parametrize("direct", [False, True])
def test_tolerances_in_turn_on_one_handle(direct):
    """Solves with different tolerances one after another on one handle:
    each must use its own states only (a state left by the previous solve
    must never be taken for one of this solve)."""
    p, Ns = 2, [4096, 1024, 16384]
    lams, Ts, u0, fs = _case(31, Ns, p)
    s = B().Solver(Ns, Ts, lams, p=p)
    s.set_schedule(256, pairs=True, direct=direct)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    for rtol in (1e-4, 1e-10, 1e-6, 1e-4, 1e-10):
        r = s.solve(f, d0, rtol=rtol)
        assert r.status == 0
        U = host(r.u)
        for j, n in enumerate(Ns):
            uo, k, rr, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j], rtol=rtol)
            assert r.cycles[j] == k, (rtol, j)
            # the residual of iterates equal to ~1e-15 differs by ~1e-15 of r_0
            assert abs(r.relres[j] - rr) <= 1e-6 * rr + 1e-13
            seg = slice(s.offsets[j], s.offsets[j + 1])
            assert relerr(U[seg], uo) <= 1e-12


@pytest.mark.parametrize("max_cycles", [0, 1, 2, 4, 5])
def test_cycle_cap(max_cycles):
    """A cap below, at and above the three cycles queued first."""
    p, Ns = 1, [2048, 512]
    lams, Ts, u0, fs = _case(32, Ns, p)
    s = B().Solver(Ns, Ts, lams, p=p)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    u = torch.full_like(f, 3.0)
    r = s.solve(f, d0, u=u, rtol=1e-12, max_cycles=max_cycles)
    assert r.status == B().TMG_NOT_CONVERGED
    U = host(u)
    for j, n in enumerate(Ns):
        assert r.cycles[j] == max_cycles
        seg = slice(s.offsets[j], s.offsets[j + 1])
        if max_cycles == 0:
            assert r.relres[j] == 1.0
            assert np.all(U[seg] == 0.0)
            continue
        uo, k, rr, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j], rtol=1e-12,
                                  max_cycles=max_cycles)
        assert k == max_cycles
        assert abs(r.relres[j] - rr) <= 1e-6 * rr + 1e-13
        assert relerr(U[seg], uo) <= 1e-12


def test_uneven_convergence_in_one_batch():
    """Instances that finish after very different numbers of cycles (the
    host queues for the slowest; cycles queued after an instance finished
    leave it untouched)."""
    p = 1
    Ns = [8192, 2, 4096, 64, 32768]
    lams = [1.0, 3.0, 200.0, 0.05, 2.0]
    Ts = [80.0, 1.0, 1.0, 0.5, 300.0]
    rng = np.random.default_rng(33)
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rng.standard_normal(n * (p + 1)) for n in Ns]
    fs[1] = np.zeros(2 * (p + 1))   # r_0 = 0 needs u0 = 0 as well
    u0[1] = 0.0
    s = B().Solver(Ns, Ts, lams, p=p)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    r = s.solve(f, d0, rtol=1e-10)
    assert r.status == 0
    U = host(r.u)
    ks = []
    for j, n in enumerate(Ns):
        seg = slice(s.offsets[j], s.offsets[j + 1])
        if j == 1:
            assert r.cycles[j] == 0 and np.all(U[seg] == 0.0)
            continue
        uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j])
        ks.append(k)
        assert r.cycles[j] == k
        assert relerr(U[seg], uo) <= 1e-12
    assert max(ks) > min(ks)


def test_solves_on_two_streams_in_turn():
    """A solve may return with cycles still queued on its stream (they do
    nothing once its instances finished).  A following solve on another
    stream resets the state those cycles read, so it must wait for them:
    both results stay the oracle's."""
    p, Ns = 3, [8192]
    lams, Ts, u0, fs = _case(34, Ns, p)
    s = B().Solver(Ns, Ts, lams, p=p)
    f1, d0 = dev(fs[0]), dev(u0)
    f2 = dev(fs[0][::-1].copy())
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ref1, k1, _, _ = core.solve(p, Ts[0], lams[0], u0[0], fs[0], rtol=1e-4)
    ref2, k2, _, _ = core.solve(p, Ts[0], lams[0], u0[0], fs[0][::-1].copy(), rtol=1e-10)
    torch.cuda.synchronize()   # inputs made on the default stream
    for _ in range(3):
        with torch.cuda.stream(s1):
            r1 = s.solve(f1, d0, rtol=1e-4)
        with torch.cuda.stream(s2):
            r2 = s.solve(f2, d0, rtol=1e-10)
        torch.cuda.synchronize()
        assert r1.cycles[0] == k1 and r2.cycles[0] == k2
        assert relerr(host(r1.u), ref1) <= 1e-12
        assert relerr(host(r2.u), ref2) <= 1e-12


def _uneven_batch(p, seed):
    """Most tiles belong to instances done after two or three cycles, the
    rest to ones that need about twelve (shuffled, so that the running
    instances of the later cycles are scattered over the batch)."""
    Ns = [4096] * 28 + [4096] * 6 + [1024, 2048, 1024, 2048, 1024, 2048]
    lams = [2e5] * 28 + [2e4] * 6 + [0.5, 10.0, 0.5, 10.0, 1.0, 3.0]
    Ts = [1.0] * 34 + [1.0, 1.0, 1.0, 1.0, 40.0, 5.0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(Ns))
    Ns, lams, Ts = ([x[i] for i in perm] for x in (Ns, lams, Ts))
    u0 = rng.uniform(-1, 1, len(Ns))
    fs = [rng.standard_normal(n * (p + 1)) for n in Ns]
    return Ns, lams, Ts, u0, fs


@pytest.mark.parametrize("precision,direct", [(0, False), (0, True), (1, False)])
def test_active_set_is_bitwise_the_full_lists(precision, direct):
    """Later cycles on the running instances' tiles only give bitwise the
    iterate, cycle counts and residuals of cycles on every tile (and the
    oracle's solve)."""
    p = 1
    Ns, lams, Ts, u0, fs = _uneven_batch(p, 35)
    s = B().Solver(Ns, Ts, lams, p=p, precision=precision)
    s.set_schedule(256, pairs=True, direct=direct)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    res = {}
    for on in (True, False, True):
        s.set_active_set(on)
        u = torch.full_like(f, 7.0)
        r = s.solve(f, d0, u=u, rtol=1e-10)
        assert r.status == 0
        res.setdefault(on, []).append((host(u), list(r.cycles), list(r.relres)))
    (Ua, ca, ra), (Ub, cb, rb) = res[True]
    (Uo, co, ro), = res[False]
    assert np.array_equal(Ua, Uo) and np.array_equal(Ub, Uo)
    assert ca == co and cb == co and ra == ro and rb == ro
    assert max(co) >= 10 and min(co) <= 3
    for j in range(len(Ns)):
        if co[j] < 10 and j % 5:
            continue
        seg = slice(s.offsets[j], s.offsets[j + 1])
        if precision == 0:
            uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], fs[j], rtol=1e-10)
            assert co[j] == k, j
            assert relerr(Uo[seg], uo) <= 1e-12
        else:
            _, km, _, _ = core.solve_mixed(p, Ts[j], lams[j], u0[j], fs[j], rtol=1e-10)
            assert abs(co[j] - km) <= 1, j
            ud = core.direct_solve(p, Ts[j], lams[j], u0[j], fs[j])
            assert relerr(Uo[seg], ud) <= 1e-8


def test_active_set_adjoint_is_bitwise_the_full_lists():
    """The same for the adjoint solve (backward in time)."""
    p = 2
    Ns, lams, Ts, u0, fs = _uneven_batch(p, 36)
    s = B().Solver(Ns, Ts, lams, p=p)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    u = torch.empty_like(f)
    r = s.solve(f, d0, u=u, rtol=1e-10)
    assert r.status == 0
    g = dev(np.random.default_rng(37).standard_normal(f.numel()))
    out = {}
    for on in (True, False):
        s.set_active_set(on)
        z = torch.full_like(f, -2.0)
        z_, dl, du, cyc, rr, st = s.adjoint_solve(g, u=u, z=z, rtol=1e-10)
        assert st == 0
        out[on] = (host(z), list(dl), list(du), list(cyc), list(rr))
    zt, zf = out[True], out[False]
    assert np.array_equal(zt[0], zf[0])
    assert zt[1:] == zf[1:]
    assert max(zf[3]) > 2 * min(zf[3])


def test_active_set_with_cycle_cap_on_two_streams():
    """Active-set lists with a cycle cap that stops the slow instances, in
    solves on two streams in turn: bitwise the full lists' results, and the
    capped instances report their cap."""
    p = 1
    Ns, lams, Ts, u0, fs = _uneven_batch(p, 38)
    s = B().Solver(Ns, Ts, lams, p=p)
    s.set_schedule(256, pairs=True, direct=True)
    f, d0 = dev(np.concatenate(fs)), dev(u0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    out = {}
    for on, st in ((True, s1), (False, s2), (True, s2), (False, s1)):
        s.set_active_set(on)
        with torch.cuda.stream(st):
            u = torch.full_like(f, 1.0)
            r = s.solve(f, d0, u=u, rtol=1e-10, max_cycles=6)
        torch.cuda.synchronize()
        out.setdefault(on, []).append((host(u), list(r.cycles), list(r.relres), r.status))
    ref = out[False][0]
    for res in out[True] + out[False][1:]:
        assert np.array_equal(res[0], ref[0])
        assert res[1:] == ref[1:]
    assert ref[3] == B().TMG_NOT_CONVERGED
    assert max(ref[1]) == 6 and min(ref[1]) <= 3


def test_batch_above_the_run_bit_limit():
    """A batch of more than 65536 instances (no run bits in the summary, so no
    active-set lists; k_publish reduces over many rounds of its work-group):
    every instance converges, and sampled ones equal their oracle solves."""
    p = 0
    B_ = 70000
    rng = np.random.default_rng(39)
    Ns = [8192 if j % 1000 == 7 else (4 if j % 3 else 256) for j in range(B_)]
    lams = list(rng.uniform(0.5, 5.0, B_))
    Ts = list(rng.uniform(0.5, 4.0, B_))
    u0 = rng.uniform(-1, 1, B_)
    f = rng.standard_normal(sum(Ns) * (p + 1))
    s = B().Solver(Ns, Ts, lams, p=p)
    r = s.solve(dev(f), dev(u0), rtol=1e-10)
    assert r.status == 0
    U = host(r.u)
    for j in list(range(0, B_, 9973)) + [7, 69007, B_ - 1]:
        seg = slice(s.offsets[j], s.offsets[j + 1])
        uo, k, _, _ = core.solve(p, Ts[j], lams[j], u0[j], f[seg], rtol=1e-10)
        assert r.cycles[j] == k, j
        assert relerr(U[seg], uo) <= 1e-12
