"""``torch.autograd.Function`` around the multigrid solve and its adjoint.

Forward: u = L(lambda)^{-1} (f + u0 v e_1), solved by ``tmg_solve``.
Backward (a loss J with dJ/du = g): the adjoint solve L^T z = g runs the
transposed multigrid cycle backward in time (``tmg_adjoint_solve``), and
    dJ/df = z,   dJ/du0 = v^T z_1,   dJ/dlambda = -sum_n z_n^T M_tau u_n,
all computed in the HIP library.

One handle serves every call of a shape (slab counts, horizons, options):
lambda is handed to the library as a device tensor (``tmg_set_lambda``
rebuilds the tables on the GPU), so a learnable lambda costs neither a
set-up nor a read-back per step.
"""
from __future__ import annotations

import torch

from .binding import Solver, TMG_OK

_cache: dict = {}


def _solver(n_slabs, T, opts, lam):
    key = (tuple(n_slabs), tuple(T), tuple(sorted(opts.items())))
    s = _cache.get(key)
    if s is None:
        if len(_cache) >= 8:
            _cache.pop(next(iter(_cache))).close()
        # the set-up's own lambda is replaced before every solve
        s = Solver(n_slabs, T, [1.0] * len(n_slabs), **opts)
        _cache[key] = s
    s.set_lambda(lam)
    return s


class TmgSolve(torch.autograd.Function):
    """TmgSolve.apply(f, u0, lam, n_slabs, T, rtol, opts) -> u.

    f: flat float64 load vectors [instance][slab][k] on the GPU; u0, lam:
    float64 tensors of length batch on the GPU; n_slabs, T: lists; opts:
    dict of ``tmg_options`` fields (p, nu1, nu2, gamma, ...)."""

    @staticmethod
    def forward(ctx, f, u0, lam, n_slabs, T, rtol, opts):
        lam_d = lam.detach().to(device=f.device, dtype=torch.float64).contiguous()
        s = _solver(n_slabs, T, opts, lam_d)
        res = s.solve(f.detach().contiguous(), u0.detach().contiguous(), rtol=rtol,
                      max_cycles=200)
        if res.status != TMG_OK:
            raise RuntimeError(f"forward solve did not converge: relres {res.relres}")
        ctx.solver = s
        ctx.rtol = rtol
        ctx.save_for_backward(res.u, lam_d)
        return res.u.clone()

    @staticmethod
    def backward(ctx, grad_u):
        u, lam_d = ctx.saved_tensors
        s = ctx.solver
        # another forward on the same handle may have changed its lambda
        s.set_lambda(lam_d)
        z, dlam, du0, _, rr, st = s.adjoint_solve(grad_u.contiguous(), u=u, rtol=ctx.rtol,
                                                  max_cycles=200)
        if st != TMG_OK:
            raise RuntimeError(f"adjoint solve did not converge: relres {rr}")
        dev = grad_u.device
        return (z, torch.tensor(du0, dtype=torch.float64, device=dev),
                torch.tensor(dlam, dtype=torch.float64, device=dev), None, None, None, None)


def solve(f, u0, lam, n_slabs, T, rtol=1e-10, **opts):
    return TmgSolve.apply(f, u0, lam, list(n_slabs), list(T), rtol, opts)
