"""ctypes wrapper around the plain-C FP64 oracle ``tmg_oracle.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Every array is a C-contiguous float64 NumPy array in slab-major layout,
coefficient ``k`` of slab ``n`` at ``n*P + k`` (``P = p + 1``).  ``f`` arguments
of the low-level calls are the *folded* right-hand side (the initial value
already added to slab 0, see :func:`fold`); :func:`solve` and
:func:`direct_solve` take the unfolded load vector and ``u0``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tmg_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libtmg_oracle.so")

_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        sig = {
            "or_tables": [_i, _d, _d, _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pd],
            "or_fold": [_i, _i64, _d, _pd, _pd],
            "or_apply": [_i, _i64, _d, _d, _i, _pd, _pd, _i],
            "or_residual": [_i, _i64, _d, _d, _i, _pd, _pd, _pd, _i],
            "or_sweeps": [_i, _i64, _d, _d, _i, _d, _i, _pd, _pd, _i],
            "or_restrict": [_i, _i64, _pd, _pd],
            "or_prolong_add": [_i, _i64, _pd, _pd],
            "or_direct": [_i, _i64, _d, _d, _i, _pd, _pd, _i],
            "or_levels": [_i, _i64, _d, _d, _i64, _i, _d, _pd, _pd],
            "or_cycles": [_i, _i64, _d, _d, _i, _i, _i, _i64, _i, _d, _i, _i, _pd, _pd, _i],
            "or_solve": [_i, _i64, _d, _d, _i, _i, _i, _i64, _i, _d, _i, _pd, _d, _i, _pd,
                         _pd, _pd, _i],
            "or_solve_mixed": [_i, _i64, _d, _d, _i, _i, _i, _i64, _i, _d, _i, _pd, _d, _i,
                               _pd, _pd, _pd],
            "or_cycle_mixed": [_i, _i64, _d, _d, _i, _i, _i, _i64, _i, _d, _i, _pd, _pd],
            "or_adjoint_rhs": [_i, _i64, _pd, _pd, _pd, _pd],
            "or_heat_fold": [_i, _i, _i64, _pd, _pd, _pd],
            "or_heat_apply": [_i, _i, _i64, _d, _pd, _pd],
            "or_heat_residual": [_i, _i, _i64, _d, _pd, _pd, _pd],
            "or_heat_sweeps": [_i, _i, _i64, _d, _d, _i, _pd, _pd],
            "or_heat_direct": [_i, _i, _i64, _d, _pd, _pd],
            "or_heat_levels": [_i, _i, _i64, _d, _i64, _i, _d, _pd],
            "or_heat_cycles": [_i, _i, _i64, _d, _i, _i, _i, _i64, _i, _d, _i, _pd, _pd],
            "or_heat_solve": [_i, _i, _i64, _d, _i, _i, _i, _i64, _i, _d, _pd, _d, _i, _pd, _pd,
                              _pd],
            "or_gradients": [_i, _i64, _d, _d, _pd, _pd, _pd, _pd],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _i
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_pd)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _dref():
    return ctypes.c_double(0.0)


@dataclass
class Opts:
    """Cycle parameters (defaults: V-cycle, 2/2 sweeps, coarsest 2 slabs,
    optimal per-level damping of Lemma chap4_lemma7)."""
    nu1: int = 2
    nu2: int = 2
    gamma: int = 1
    n_coarse: int = 2
    omega_mode: int = 0      # 0 optimal per level, 1 fixed
    omega: float = 0.5       # used when omega_mode == 1


def tables(p: int, tau: float, lam: float):
    """K, M, N, A, alpha, omega*, R1T, R2T for one slab of length tau."""
    P = p + 1
    K, M, N, A, R1T, R2T = (np.zeros((P, P)) for _ in range(6))
    a, w = _dref(), _dref()
    rc = lib().or_tables(p, tau, lam, _p(K), _p(M), _p(N), _p(A), ctypes.byref(a),
                         ctypes.byref(w), _p(R1T), _p(R2T))
    assert rc == 0
    return dict(K=K, M=M, N=N, A=A, alpha=a.value, omega=w.value, R1T=R1T, R2T=R2T)


def fold(p: int, u0: float, f) -> np.ndarray:
    f = _c(f)
    out = np.empty_like(f)
    lib().or_fold(p, f.size // (p + 1), float(u0), _p(f), _p(out))
    return out


def apply(p: int, tau: float, lam: float, u, trans: bool = False,
          periodic: bool = False) -> np.ndarray:
    """L u (or L^T u); periodic: the circulant system u(0) = u(T)."""
    u = _c(u)
    out = np.empty_like(u)
    lib().or_apply(p, u.size // (p + 1), tau, lam, int(trans), _p(u), _p(out), int(periodic))
    return out


def residual(p: int, tau: float, lam: float, f, u, trans: bool = False,
             periodic: bool = False) -> np.ndarray:
    f, u = _c(f), _c(u)
    r = np.empty_like(f)
    lib().or_residual(p, f.size // (p + 1), tau, lam, int(trans), _p(f), _p(u), _p(r),
                      int(periodic))
    return r


def sweeps(p: int, tau: float, lam: float, f, u, nsweep: int, omega: float = 0.0,
           trans: bool = False, periodic: bool = False) -> np.ndarray:
    """nsweep damped block Jacobi steps from u (omega <= 0: optimal omega*)."""
    f = _c(f)
    u = _c(u).copy()
    lib().or_sweeps(p, f.size // (p + 1), tau, lam, int(trans), omega, nsweep, _p(f), _p(u),
                    int(periodic))
    return u


def restrict(p: int, r) -> np.ndarray:
    r = _c(r)
    nc = r.size // (p + 1) // 2
    rc = np.empty(nc * (p + 1))
    lib().or_restrict(p, nc, _p(r), _p(rc))
    return rc


def prolong_add(p: int, e, u) -> np.ndarray:
    e = _c(e)
    u = _c(u).copy()
    lib().or_prolong_add(p, e.size // (p + 1), _p(e), _p(u))
    return u


def direct(p: int, tau: float, lam: float, f, trans: bool = False,
           periodic: bool = False) -> np.ndarray:
    """Exact solve of L u = f (folded f) by forward substitution, or of
    L^T z = g by backward substitution; periodic: of the circulant system."""
    f = _c(f)
    u = np.empty_like(f)
    lib().or_direct(p, f.size // (p + 1), tau, lam, int(trans), _p(f), _p(u), int(periodic))
    return u


def direct_solve(p: int, T: float, lam: float, u0: float, f) -> np.ndarray:
    """The plain definition: sequential DG time stepping from u0."""
    f = fold(p, u0, f)
    return direct(p, T / (f.size // (p + 1)), lam, f)


def levels(p: int, N: int, T: float, lam: float, opts: Opts = Opts()):
    a = np.zeros(64)
    w = np.zeros(64)
    n = lib().or_levels(p, N, T, lam, opts.n_coarse, opts.omega_mode, opts.omega, _p(a), _p(w))
    assert n > 0
    return a[:n].copy(), w[:n].copy()


def cycles(p: int, T: float, lam: float, f, u, ncyc: int, opts: Opts = Opts(),
           trans: bool = False, periodic: bool = False) -> np.ndarray:
    """ncyc reference cycles on the folded system from initial guess u."""
    f = _c(f)
    u = _c(u).copy()
    rc = lib().or_cycles(p, f.size // (p + 1), T, lam, opts.nu1, opts.nu2, opts.gamma,
                         opts.n_coarse, opts.omega_mode, opts.omega, int(trans), ncyc, _p(f),
                         _p(u), int(periodic))
    assert rc == 0
    return u


def solve_folded(p: int, T: float, lam: float, f, rtol: float = 1e-10, max_cycles: int = 200,
                 opts: Opts = Opts(), trans: bool = False, periodic: bool = False):
    """Reference multigrid solve from zero; returns (u, cycles, relres, hist)."""
    f = _c(f)
    u = np.empty_like(f)
    hist = np.zeros(max_cycles + 1)
    rr = _dref()
    k = lib().or_solve(p, f.size // (p + 1), T, lam, opts.nu1, opts.nu2, opts.gamma,
                       opts.n_coarse, opts.omega_mode, opts.omega, int(trans), _p(f), rtol,
                       max_cycles, _p(u), ctypes.byref(rr), _p(hist), int(periodic))
    assert k >= 0
    return u, k, rr.value, hist[:k + 1].copy()


def solve(p: int, T: float, lam: float, u0: float, f, rtol: float = 1e-10,
          max_cycles: int = 200, opts: Opts = Opts()):
    return solve_folded(p, T, lam, fold(p, u0, f), rtol, max_cycles, opts)


def solve_mixed(p: int, T: float, lam: float, u0: float, f, rtol: float = 1e-10,
                max_cycles: int = 200, opts: Opts = Opts(), lb64: int = -1):
    """FP32-inner / FP64-outer defect-correction reference.  lb64: first level
    whose visits run in FP64 arithmetic from FP32 operands (-1: the coarsest
    level only)."""
    f = fold(p, u0, f)
    u = np.empty_like(f)
    hist = np.zeros(max_cycles + 1)
    rr = _dref()
    k = lib().or_solve_mixed(p, f.size // (p + 1), T, lam, opts.nu1, opts.nu2, opts.gamma,
                             opts.n_coarse, opts.omega_mode, opts.omega, lb64, _p(f), rtol,
                             max_cycles, _p(u), ctypes.byref(rr), _p(hist))
    assert k >= 0
    return u, k, rr.value, hist[:k + 1].copy()


def cycle_mixed(p: int, T: float, lam: float, r, opts: Opts = Opts(), lb64: int = -1):
    """One FP32-inner cycle on L e = r (folded r, rounded to FP32) from e = 0:
    the inner correction of the defect correction, returned in double."""
    r = _c(r)
    e = np.empty_like(r)
    rc = lib().or_cycle_mixed(p, r.size // (p + 1), T, lam, opts.nu1, opts.nu2, opts.gamma,
                              opts.n_coarse, opts.omega_mode, opts.omega, lb64, _p(r), _p(e))
    assert rc == 0
    return e


def adjoint_rhs(p: int, u, y):
    """g_n = (w_n - y_n) psi(t_n^-) and J = 1/2 sum (w_n - y_n)^2."""
    u, y = _c(u), _c(y)
    g = np.empty_like(u)
    J = _dref()
    lib().or_adjoint_rhs(p, u.size // (p + 1), _p(u), _p(y), _p(g), ctypes.byref(J))
    return g, J.value


def gradients(p: int, tau: float, lam: float, u, z):
    """(dJ/dlambda, dJ/du0) from the forward solution u and adjoint z."""
    u, z = _c(u), _c(z)
    dl, du = _dref(), _dref()
    lib().or_gradients(p, u.size // (p + 1), tau, lam, _p(u), _p(z), ctypes.byref(dl),
                       ctypes.byref(du))
    return dl.value, du.value


# --------------------------------------------------------------------------
# space-time heat equation u_t - u_xx = f on (0,1), u = 0 at x = 0, 1
# (arrays [point][slab][k], nx interior points of h = 1/(nx+1))
# --------------------------------------------------------------------------

def heat_fold(p: int, nx: int, u0, f) -> np.ndarray:
    f, u0 = _c(f), _c(u0)
    out = np.empty_like(f)
    lib().or_heat_fold(p, nx, f.size // (nx * (p + 1)), _p(u0), _p(f), _p(out))
    return out


def heat_apply(p: int, nx: int, tau: float, u) -> np.ndarray:
    u = _c(u)
    out = np.empty_like(u)
    lib().or_heat_apply(p, nx, u.size // (nx * (p + 1)), tau, _p(u), _p(out))
    return out


def heat_residual(p: int, nx: int, tau: float, f, u) -> np.ndarray:
    f, u = _c(f), _c(u)
    r = np.empty_like(f)
    lib().or_heat_residual(p, nx, f.size // (nx * (p + 1)), tau, _p(f), _p(u), _p(r))
    return r


def heat_sweeps(p: int, nx: int, tau: float, f, u, nsweep: int, omega: float = 0.0) -> np.ndarray:
    f = _c(f)
    u = _c(u).copy()
    lib().or_heat_sweeps(p, nx, f.size // (nx * (p + 1)), tau, omega, nsweep, _p(f), _p(u))
    return u


def heat_direct(p: int, nx: int, tau: float, f) -> np.ndarray:
    f = _c(f)
    u = np.empty_like(f)
    lib().or_heat_direct(p, nx, f.size // (nx * (p + 1)), tau, _p(f), _p(u))
    return u


def heat_levels(p: int, nx: int, N: int, T: float, opts: Opts = Opts()) -> np.ndarray:
    w = np.zeros(64)
    n = lib().or_heat_levels(p, nx, N, T, opts.n_coarse, opts.omega_mode, opts.omega, _p(w))
    assert n > 0
    return w[:n].copy()


def heat_cycles(p: int, nx: int, T: float, f, u, ncyc: int, opts: Opts = Opts()) -> np.ndarray:
    f = _c(f)
    u = _c(u).copy()
    rc = lib().or_heat_cycles(p, nx, f.size // (nx * (p + 1)), T, opts.nu1, opts.nu2,
                              opts.gamma, opts.n_coarse, opts.omega_mode, opts.omega, ncyc,
                              _p(f), _p(u))
    assert rc == 0
    return u


def heat_solve_folded(p: int, nx: int, T: float, f, rtol: float = 1e-10, max_cycles: int = 200,
                      opts: Opts = Opts()):
    f = _c(f)
    u = np.empty_like(f)
    hist = np.zeros(max_cycles + 1)
    rr = _dref()
    k = lib().or_heat_solve(p, nx, f.size // (nx * (p + 1)), T, opts.nu1, opts.nu2, opts.gamma,
                            opts.n_coarse, opts.omega_mode, opts.omega, _p(f), rtol, max_cycles,
                            _p(u), ctypes.byref(rr), _p(hist))
    assert k >= 0
    return u, k, rr.value, hist[:k + 1].copy()
