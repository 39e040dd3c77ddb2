"""``torch.autograd.Function`` around the multigrid solve and its adjoint.

Forward: u = L(lambda)^{-1} (f + u0 v e_1), solved by ``tmg_solve``.
Backward (a loss J with dJ/du = g): the adjoint solve L^T z = g runs the
transposed multigrid cycle backward in time (``tmg_adjoint_solve``), and
    dJ/df = z,   dJ/du0 = v^T z_1,   dJ/dlambda = -sum_n z_n^T M_tau u_n,
all computed in the HIP library.
"""
from __future__ import annotations

import torch

from .binding import Solver, TMG_OK

_cache: dict = {}


def _solver(n_slabs, T, lam, opts):
    key = (tuple(n_slabs), tuple(T), tuple(lam), tuple(sorted(opts.items())))
    s = _cache.get(key)
    if s is None:
        if len(_cache) > 8:
            _cache.clear()
        s = Solver(n_slabs, T, lam, **opts)
        _cache[key] = s
    return s


class TmgSolve(torch.autograd.Function):
    """TmgSolve.apply(f, u0, lam, n_slabs, T, rtol, opts) -> u.

    f: flat float64 load vectors [instance][slab][k] on the GPU; u0, lam:
    float64 tensors of length batch; n_slabs, T: lists; opts: dict of
    ``tmg_options`` fields (p, nu1, nu2, gamma, ...)."""

    @staticmethod
    def forward(ctx, f, u0, lam, n_slabs, T, rtol, opts):
        lam_l = [float(x) for x in lam.detach().cpu().tolist()]
        s = _solver(n_slabs, T, lam_l, opts)
        res = s.solve(f.detach().contiguous(), u0.detach().contiguous(), rtol=rtol,
                      max_cycles=200)
        if res.status != TMG_OK:
            raise RuntimeError(f"forward solve did not converge: relres {res.relres}")
        ctx.solver = s
        ctx.rtol = rtol
        ctx.save_for_backward(res.u)
        return res.u.clone()

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        s = ctx.solver
        z, dlam, du0, _, rr, st = s.adjoint_solve(grad_u.contiguous(), u=u, rtol=ctx.rtol,
                                                  max_cycles=200)
        if st != TMG_OK:
            raise RuntimeError(f"adjoint solve did not converge: relres {rr}")
        dev = grad_u.device
        return (z, torch.tensor(du0, dtype=torch.float64, device=dev),
                torch.tensor(dlam, dtype=torch.float64, device=dev), None, None, None, None)


def solve(f, u0, lam, n_slabs, T, rtol=1e-10, **opts):
    return TmgSolve.apply(f, u0, lam, list(n_slabs), list(T), rtol, opts)
