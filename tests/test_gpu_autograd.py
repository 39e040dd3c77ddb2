"""GPU: the autograd function (forward multigrid solve, backward adjoint
multigrid solve) against finite differences and torch.autograd.gradcheck.

The loss is J = 1/2 sum_n (w_n - y_n)^2 with w_n = u_n(t_n^-) = sum_k u_n[k]
(the adjoint batch's loss).  Forward solves for the differences run to a relative
residual of 1e-13 so that solve error times J/h stays below the check."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import core  # noqa: E402

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def A():
    from paper_1409_5254_amd import autograd
    return autograd


def loss(u, y, P):
    w = u.view(-1, P).sum(dim=1)
    return 0.5 * ((w - y) ** 2).sum()


@pytest.mark.parametrize("p", [1, 2])
def test_gradients_match_central_differences(p):
    rng = np.random.default_rng(80 + p)
    B, N, T = 3, 256, 4.0
    P = p + 1
    f = torch.tensor(rng.standard_normal(B * N * P) * 0.1, dtype=torch.float64, device=DEV,
                     requires_grad=True)
    u0 = torch.tensor(rng.uniform(0.5, 1.5, B), dtype=torch.float64, device=DEV,
                      requires_grad=True)
    lam = torch.tensor(rng.uniform(0.1, 10.0, B), dtype=torch.float64, device=DEV,
                       requires_grad=True)
    y = torch.tensor(rng.standard_normal(B * N), dtype=torch.float64, device=DEV)
    u = A().solve(f, u0, lam, [N] * B, [T] * B, rtol=1e-13, p=p)
    J = loss(u, y, P)
    J.backward()
    h = 1e-6

    def Jat(f_, u0_, lam_):
        with torch.no_grad():
            return loss(A().solve(f_, u0_, lam_, [N] * B, [T] * B, rtol=1e-13, p=p), y, P).item()

    with torch.no_grad():
        for j in range(B):
            e = torch.zeros(B, dtype=torch.float64, device=DEV)
            e[j] = h
            fd_l = (Jat(f, u0, lam + e) - Jat(f, u0, lam - e)) / (2 * h)
            fd_u = (Jat(f, u0 + e, lam) - Jat(f, u0 - e, lam)) / (2 * h)
            assert lam.grad[j].item() == pytest.approx(fd_l, rel=1e-5, abs=1e-9)
            assert u0.grad[j].item() == pytest.approx(fd_u, rel=1e-5, abs=1e-9)
        d = torch.tensor(rng.standard_normal(B * N * P), dtype=torch.float64, device=DEV)
        fd_f = (Jat(f + h * d, u0, lam) - Jat(f - h * d, u0, lam)) / (2 * h)
        assert (f.grad * d).sum().item() == pytest.approx(fd_f, rel=1e-5)


def test_adjoint_against_oracle_gradients():
    """Backward pass of the autograd function against the oracle's adjoint
    gradients (direct forward and backward substitution)."""
    rng = np.random.default_rng(90)
    p, N, T, lam, u0 = 2, 2048, 100.0, 3.0, 1.0
    P = p + 1
    fn = rng.standard_normal(N * P) * 0.01
    yn = rng.standard_normal(N)
    f = torch.tensor(fn, dtype=torch.float64, device=DEV, requires_grad=True)
    u0t = torch.tensor([u0], dtype=torch.float64, device=DEV, requires_grad=True)
    lt = torch.tensor([lam], dtype=torch.float64, device=DEV, requires_grad=True)
    u = A().solve(f, u0t, lt, [N], [T], rtol=1e-13, p=p)
    loss(u, torch.tensor(yn, dtype=torch.float64, device=DEV), P).backward()
    ud = core.direct_solve(p, T, lam, u0, fn)
    g, _ = core.adjoint_rhs(p, ud, yn)
    z = core.direct(p, T / N, lam, g, trans=True)
    dl, du = core.gradients(p, T / N, lam, ud, z)
    zg = f.grad.detach().cpu().numpy()
    assert np.max(np.abs(zg - z)) <= 1e-9 * np.max(np.abs(z))
    assert lt.grad.item() == pytest.approx(dl, rel=1e-9)
    assert u0t.grad.item() == pytest.approx(du, rel=1e-9)


def test_gradcheck_tiny():
    """torch.autograd.gradcheck at a tiny FP64 size (N = 8 slabs)."""
    rng = np.random.default_rng(91)
    p, N, T = 1, 8, 2.0
    f = torch.tensor(rng.standard_normal(N * 2), dtype=torch.float64, device=DEV,
                     requires_grad=True)
    u0 = torch.tensor([0.7], dtype=torch.float64, device=DEV, requires_grad=True)
    lam = torch.tensor([1.3], dtype=torch.float64, device=DEV, requires_grad=True)
    fn = lambda f_, u0_, l_: A().solve(f_, u0_, l_, [N], [T], rtol=1e-13, p=p)
    assert torch.autograd.gradcheck(fn, (f, u0, lam), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_learnable_lambda_steps_on_one_handle():
    """Five gradient steps on a learnable lambda through the autograd
    function: one handle serves every step (tmg_set_lambda rebuilds its
    tables on the GPU), and every step's gradients equal the oracle's
    (direct forward and backward substitution at the current lambda)."""
    ag = A()
    rng = np.random.default_rng(92)
    p, N, T, B = 2, 1024, 20.0, 2
    P = p + 1
    fn = rng.standard_normal(B * N * P) * 0.01
    yn = rng.standard_normal(B * N)
    f = torch.tensor(fn, dtype=torch.float64, device=DEV)
    u0 = torch.tensor([1.0, 0.5], dtype=torch.float64, device=DEV)
    lam = torch.tensor([2.0, 0.7], dtype=torch.float64, device=DEV, requires_grad=True)
    y = torch.tensor(yn, dtype=torch.float64, device=DEV)
    opt = torch.optim.SGD([lam], lr=1e-3)
    ag._cache.clear()
    handles = set()
    for step in range(5):
        opt.zero_grad()
        u = ag.solve(f, u0, lam, [N] * B, [T] * B, rtol=1e-13, p=p)
        loss(u, y, P).backward()
        handles.update(id(s) for s in ag._cache.values())
        lam_now = lam.detach().cpu().numpy()
        for j in range(B):
            sl = slice(j * N * P, (j + 1) * N * P)
            ud = core.direct_solve(p, T, lam_now[j], float(u0[j]), fn[sl])
            g, _ = core.adjoint_rhs(p, ud, yn[j * N:(j + 1) * N])
            z = core.direct(p, T / N, lam_now[j], g, trans=True)
            dl, _ = core.gradients(p, T / N, lam_now[j], ud, z)
            assert lam.grad[j].item() == pytest.approx(dl, rel=1e-9), (step, j)
        opt.step()
    assert len(ag._cache) == 1 and len(handles) == 1


@pytest.mark.parametrize("gamma", [1, 2])
def test_set_lambda_equals_setup(gamma):
    """A handle set up with lambda_1 and switched to lambda_2 by
    tmg_set_lambda solves (forward and adjoint, with gradients) to the same
    bits as a handle set up with lambda_2: the device rebuilds the tables to
    the host's bits."""
    from paper_1409_5254_amd.binding import Solver
    rng = np.random.default_rng(93)
    p, Ns = 3, [4096, 512, 8192]
    P = p + 1
    Ts = [10.0, 3.0, 40.0]
    lam1 = [1.0, 2.0, 3.0]
    lam2 = [25.0, 0.01, 4e3]
    f = torch.tensor(rng.standard_normal(sum(Ns) * P) * 0.1, dtype=torch.float64, device=DEV)
    u0 = torch.tensor([1.0, -1.0, 0.3], dtype=torch.float64, device=DEV)
    a = Solver(Ns, Ts, lam1, p=p, gamma=gamma)
    a.set_lambda(torch.tensor(lam2, dtype=torch.float64, device=DEV))
    b = Solver(Ns, Ts, lam2, p=p, gamma=gamma)
    ra = a.solve(f, u0, rtol=1e-10)
    rb = b.solve(f, u0, rtol=1e-10)
    assert ra.cycles == rb.cycles and ra.status == rb.status == 0
    assert torch.equal(ra.u, rb.u)
    g = torch.tensor(rng.standard_normal(sum(Ns) * P), dtype=torch.float64, device=DEV)
    za = a.adjoint_solve(g, u=ra.u, rtol=1e-10)
    zb = b.adjoint_solve(g, u=rb.u, rtol=1e-10)
    assert torch.equal(za[0], zb[0]) and za[1] == zb[1] and za[2] == zb[2]
    for j in range(len(Ns)):
        for lev in range(3):
            assert a.level_info(j, lev) == b.level_info(j, lev)
    a.close()
    b.close()


def test_set_lambda_invalid_is_nonfinite():
    from paper_1409_5254_amd.binding import Solver, TmgError
    s = Solver([1024], [1.0], [1.0], p=1)
    f = torch.ones(2048, dtype=torch.float64, device=DEV)
    u0 = torch.ones(1, dtype=torch.float64, device=DEV)
    s.set_lambda(torch.tensor([-1.0], dtype=torch.float64, device=DEV))
    with pytest.raises(TmgError) as e:
        s.solve(f, u0)
    assert e.value.code == -7
    s.set_lambda(torch.tensor([1.0], dtype=torch.float64, device=DEV))
    assert s.solve(f, u0).status == 0
    s.close()


@pytest.mark.parametrize("p", [1, 3])
def test_gradient_reduction_deterministic_and_bounded(p):
    """The two-stage gradient reduction over one long instance (2^22 slabs):
    repeated backward passes give the same bits, and dlambda is within the
    summation bound of the oracle's value (FP64 sums of 2^22 P terms in a
    different order: |error| <= 1e-12 |dl| + 16 eps tau sum |z_n M u_n|)."""
    from paper_1409_5254_amd.binding import Solver
    rng = np.random.default_rng(94 + p)
    N, T, lam = 1 << 22, 1000.0, 1.0
    P = p + 1
    s = Solver([N], [T], [lam], p=p)
    f = torch.tensor(rng.standard_normal(N * P) * 1e-3, dtype=torch.float64, device=DEV)
    g = torch.tensor(rng.standard_normal(N * P), dtype=torch.float64, device=DEV)
    u0 = torch.ones(1, dtype=torch.float64, device=DEV)
    u = s.solve(f, u0, rtol=1e-12).u
    outs = [s.adjoint_solve(g, u=u, rtol=1e-12) for _ in range(3)]
    assert all(o[1] == outs[0][1] and o[2] == outs[0][2] for o in outs)
    z = outs[0][0]
    un, zn = u.cpu().numpy(), z.cpu().numpy()
    dlo, du0o = core.gradients(p, T / N, lam, un, zn)
    w = np.tile(1.0 / (2.0 * np.arange(P) + 1.0), N)
    bound = 1e-12 * abs(dlo) + 16 * np.finfo(float).eps * (T / N) * np.sum(np.abs(zn * un * w))
    assert abs(outs[0][1][0] - dlo) <= bound
    assert outs[0][2][0] == pytest.approx(du0o, rel=1e-14)
    s.close()
