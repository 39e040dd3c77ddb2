"""The entry point that allocates nothing (tmg_solve_noalloc) against the
handle-based tmg_solve and the FP64 oracle.

tmg_solve_noalloc runs the same kernels as tmg_solve with the default
schedule, launched kernel by kernel instead of from captured graphs, on
buffers carved out of the library's static scratch array; the iterates are
therefore bitwise those of tmg_solve (same cycle count), and within the
1e-12 parity bar of the oracle's multigrid solve.  Consecutive calls reuse
the scratch with the previous call's contents in it: the second call of
each pair is smaller (and of another degree), so any buffer it read before
writing would carry the first call's values.
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


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def case(p, log2n, lam, seed):
    N = 1 << log2n
    T = 2.0 * N / 1024.0
    inst = gen.fourier_scalar(p, N=N, T=T).instances[0]
    f = np.asarray(inst.f)
    rng = np.random.default_rng(seed)
    f = f + 0.1 * rng.standard_normal(f.size) * np.max(np.abs(f))
    return N, T, lam, 1.0, f


def run_pair(p, N, T, lam, u0, f, oracle=True, **opts):
    b = B()
    fd = torch.as_tensor(f, dtype=torch.float64, device=DEV)
    u0d = torch.tensor([u0], dtype=torch.float64, device=DEV)
    print(f"noalloc solve p={p} N={N} lam={lam} opts={opts}", flush=True)
    r = b.solve_noalloc(N, T, lam, fd, u0d, rtol=1e-10, max_cycles=200, p=p, **opts)
    torch.cuda.synchronize()
    s = b.Solver([N], [T], [lam], p=p, **opts)
    # the entry point runs a W-cycle's bottom visits as the recursion (its
    # scratch has no room for their dense operator): so does the reference
    s.set_dense_bottom(False)
    ref = s.solve(fd, u0d, rtol=1e-10, max_cycles=200)
    torch.cuda.synchronize()
    un, uh = r.u.cpu().numpy(), ref.u.cpu().numpy()
    s.close()
    assert r.status == ref.status == 0, (r.status, ref.status)
    assert r.cycles == ref.cycles, (r.cycles, ref.cycles)
    assert r.relres == ref.relres
    assert np.array_equal(un, uh), relerr(un, uh)
    if oracle:
        uo, k, _, _ = core.solve(p, T, lam, u0, f, opts=core.Opts(**{
            k: v for k, v in opts.items() if k in ("nu1", "nu2", "gamma", "n_coarse")}))
        assert r.cycles[0] == k
        assert relerr(un, uo) <= TOL
    return r


def test_two_calls_second_smaller():
    """A streaming-level solve (p = 3, N = 2^15), then a smaller one of
    another degree (p = 1, N = 2^12) in the same scratch."""
    N, T, lam, u0, f = case(3, 15, 1.0, 1)
    run_pair(3, N, T, lam, u0, f)
    N, T, lam, u0, f = case(1, 12, 4.0, 2)
    run_pair(1, N, T, lam, u0, f)


def test_calls_whole_bottom_w_cycle_and_largest():
    """An instance the bottom kernel holds whole, a W-cycle, the largest
    size the call takes (N * P = 2^21), then a small one again."""
    N, T, lam, u0, f = case(2, 8, 2.0, 3)
    run_pair(2, N, T, lam, u0, f)
    N, T, lam, u0, f = case(1, 13, 1.0, 4)
    run_pair(1, N, T, lam, u0, f, gamma=2)
    N, T, lam, u0, f = case(3, 19, 1.0, 5)
    run_pair(3, N, T, lam, u0, f, oracle=False)
    N, T, lam, u0, f = case(0, 10, 3.0, 6)
    run_pair(0, N, T, lam, u0, f)


def test_too_large_is_rejected():
    """Above TMG_NOALLOC_MAX_UNKNOWNS coefficients the call returns
    TMG_ERR_SIZE before any device work."""
    b = B()
    N = 1 << 20
    f = torch.zeros(N * 4, dtype=torch.float64, device=DEV)
    u0 = torch.ones(1, dtype=torch.float64, device=DEV)
    with pytest.raises(b.TmgError) as e:
        b.solve_noalloc(N, 1.0, 1.0, f, u0, p=3)
    assert e.value.code == -2
