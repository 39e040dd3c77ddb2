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
