"""ctypes binding of ``libtmg.so`` (the C ABI declared in ``include/tmg.h``).

Argument marshalling only: every step of the solve runs in the HIP library.
Tensors are passed as device pointers (float64, contiguous, on the current
HIP device); the stream is torch's current stream.  There is no CPU
fallback: if the library is not built, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libtmg.so")

TMG_OK = 0
TMG_NOT_CONVERGED = 1
ERRORS = {
    -1: "TMG_ERR_INVALID", -2: "TMG_ERR_SIZE", -3: "TMG_ERR_OMEGA", -4: "TMG_ERR_PARAM",
    -5: "TMG_ERR_OOM", -6: "TMG_ERR_HIP", -7: "TMG_ERR_NONFINITE", -8: "TMG_ERR_DIVERGED",
    -9: "TMG_ERR_UNSUPPORTED", -10: "TMG_ERR_INTERNAL",
}
MAX_DEGREE = 20
MAX_TUNED_DEGREE = 5

# every symbol the header declares
SYMBOLS = ["tmg_default_options", "tmg_setup", "tmg_vcycle", "tmg_solve", "tmg_adjoint_solve",
           "tmg_autotune", "tmg_set_schedule", "tmg_set_active_set",
           "tmg_set_dense_bottom", "tmg_destroy", "tmg_error_string", "tmg_last_hip_error", "tmg_level_info",
           "tmg_level_size", "tmg_op_down", "tmg_op_up", "tmg_op_fused", "tmg_op_fused2",
           "tmg_op_coarse_solve",
           "tmg_op_residual_norm", "tmg_solve_noalloc", "tmg_op_down32", "tmg_op_up32",
           "tmg_op_mix", "tmg_set_lambda", "tmg_heat_setup", "tmg_heat_vcycle",
           "tmg_heat_solve", "tmg_heat_destroy", "tmg_heat_last_hip_error",
           "tmg_heat_set_mode_solve"]


class TmgError(RuntimeError):
    def __init__(self, code: int, where: str, hip: int = 0):
        self.code = code
        msg = f"{where}: {ERRORS.get(code, code)} ({error_string(code)})"
        if hip:
            msg += f", hipError {hip}"
        super().__init__(msg)


class Options(ctypes.Structure):
    """Mirror of ``tmg_options``."""
    _fields_ = [("p", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("gamma", ctypes.c_int), ("n_coarse", ctypes.c_int64),
                ("omega_mode", ctypes.c_int), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int), ("schedule", ctypes.c_int),
                ("periodic", ctypes.c_int)]

    @classmethod
    def make(cls, **kw) -> "Options":
        o = cls()
        lib().tmg_default_options(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise AttributeError(k)
            setattr(o, k, v)
        return o


_lib = None
_i, _i64, _d, _vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"HIP library not built: {_LIB_PATH} "
                               "(run python -m paper_1409_5254_amd.build)")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "tmg_default_options": (None, [_vp]),
            "tmg_setup": (_i, [P(_vp), _i, P(_i64), P(_d), P(_d), _vp, _vp]),
            "tmg_vcycle": (_i, [_vp, _vp, _vp, _vp, _vp]),
            "tmg_solve": (_i, [_vp, _vp, _vp, _vp, _d, _i, P(_i), P(_d), _vp]),
            "tmg_adjoint_solve": (_i, [_vp, _vp, _vp, _vp, _d, _i, P(_d), P(_d), P(_i), P(_d),
                                       _vp]),
            "tmg_autotune": (_i, [_vp, _vp, _vp, _vp, P(_i64), P(_i), P(_i), P(_i), P(_i), _vp]),
            "tmg_set_schedule": (_i, [_vp, _i64, _i, _i, _i, _i, _vp]),
            "tmg_set_active_set": (_i, [_vp, _i]),
            "tmg_set_dense_bottom": (_i, [_vp, _i, _vp]),
            "tmg_set_lambda": (_i, [_vp, _vp, _vp]),
            "tmg_destroy": (_i, [_vp]),
            "tmg_error_string": (ctypes.c_char_p, [_i]),
            "tmg_last_hip_error": (_i, [_vp]),
            "tmg_level_info": (_i, [_vp, _i, _i, P(_i64), P(_d), P(_d)]),
            "tmg_level_size": (_i64, [_vp, _i]),
            "tmg_op_down": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_up": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_fused": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_fused2": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_coarse_solve": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
            "tmg_op_residual_norm": (_i, [_vp, _i, _vp, _vp, _vp, P(_d), _vp]),
            "tmg_op_down32": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_up32": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
            "tmg_op_mix": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "tmg_heat_setup": (_i, [P(_vp), _i64, _i, _d, _vp, _vp]),
            "tmg_heat_vcycle": (_i, [_vp, _vp, _vp, _vp, _vp]),
            "tmg_heat_solve": (_i, [_vp, _vp, _vp, _vp, _d, _i, P(_i), P(_d), _vp]),
            "tmg_heat_destroy": (_i, [_vp]),
            "tmg_heat_last_hip_error": (_i, [_vp]),
            "tmg_heat_set_mode_solve": (_i, [_vp, _i]),
            "tmg_solve_noalloc": (_i, [_i64, _d, _d, _vp, _vp, _vp, _vp, _d, _i, P(_i), P(_d),
                                       _vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().tmg_error_string(code).decode()


def _ptr(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _ptr32(t):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def solve_noalloc(n_slabs, T, lam, f, u0, u=None, rtol=1e-10, max_cycles=100, **opts):
    """One instance solved by ``tmg_solve_noalloc`` (no handle; the library's
    static scratch holds every buffer beyond f, u0 and u).  Returns a
    SolveResult; raises TmgError on an error code."""
    o = Options.make(**opts)
    if u is None:
        u = torch.empty_like(f)
    cyc = (ctypes.c_int * 1)()
    rr = (ctypes.c_double * 1)()
    rc = lib().tmg_solve_noalloc(int(n_slabs), float(T), float(lam), ctypes.byref(o), _ptr(f),
                                 _ptr(u0), _ptr(u), rtol, max_cycles, cyc, rr, _stream())
    if rc < 0:
        raise TmgError(rc, "tmg_solve_noalloc")
    return SolveResult(u, list(cyc), list(rr), rc)


@dataclass
class SolveResult:
    u: torch.Tensor
    cycles: list
    relres: list
    status: int


class Solver:
    """One handle: `batch` instances with n_slabs[j] slabs on (0, T[j]] and
    decay rate lam[j].  Arrays are flat float64 device tensors laid out
    [instance][slab][k]."""

    def __init__(self, n_slabs, T, lam, **opts):
        n_slabs = [int(n) for n in n_slabs]
        self.batch = len(n_slabs)
        self.n_slabs = n_slabs
        self.T = [float(x) for x in T]
        self.lam = [float(x) for x in lam]
        self.opts = Options.make(**opts)
        self.P = self.opts.p + 1
        self.size = sum(n_slabs) * self.P
        self.offsets = [0]
        for n in n_slabs:
            self.offsets.append(self.offsets[-1] + n * self.P)
        h = ctypes.c_void_p()
        arr64 = (ctypes.c_int64 * self.batch)(*n_slabs)
        arrT = (ctypes.c_double * self.batch)(*self.T)
        arrL = (ctypes.c_double * self.batch)(*self.lam)
        rc = lib().tmg_setup(ctypes.byref(h), self.batch, arr64, arrT, arrL,
                             ctypes.byref(self.opts), _stream())
        if rc != TMG_OK:
            raise TmgError(rc, "tmg_setup")
        self._h = h

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().tmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, where):
        if rc < 0:
            raise TmgError(rc, where, lib().tmg_last_hip_error(self._h))
        return rc

    # -- whole solves ----------------------------------------------------
    def solve(self, f, u0, u=None, rtol=1e-10, max_cycles=100) -> SolveResult:
        if u is None:
            u = torch.empty_like(f)
        cyc = (ctypes.c_int * self.batch)()
        rr = (ctypes.c_double * self.batch)()
        rc = lib().tmg_solve(self._h, _ptr(f), _ptr(u0), _ptr(u), rtol, max_cycles, cyc, rr,
                             _stream())
        self._check(rc, "tmg_solve")
        return SolveResult(u, list(cyc), list(rr), rc)

    def autotune(self, f, u0, u):
        """Pick the fastest schedule on (f, u0); u is overwritten.  Returns
        dict(bottom_cap, pairs, span, span_after, direct)."""
        cap = ctypes.c_int64()
        pairs = ctypes.c_int()
        span = ctypes.c_int()
        after = ctypes.c_int()
        direct = ctypes.c_int()
        self._check(lib().tmg_autotune(self._h, _ptr(f), _ptr(u0), _ptr(u), ctypes.byref(cap),
                                       ctypes.byref(pairs), ctypes.byref(span),
                                       ctypes.byref(after), ctypes.byref(direct), _stream()),
                    "tmg_autotune")
        return dict(bottom_cap=cap.value, pairs=bool(pairs.value), span=span.value,
                    span_after=after.value, direct=bool(direct.value))

    def set_schedule(self, bottom_cap, pairs=True, span=0, span_after=2, direct=False):
        """Install a schedule without timing (see autotune)."""
        self._check(lib().tmg_set_schedule(self._h, int(bottom_cap), int(bool(pairs)), int(span),
                                           int(span_after), int(bool(direct)), _stream()),
                    "tmg_set_schedule")

    def set_lambda(self, lam):
        """New decay rates from a float64 device tensor of length batch; the
        tables are rebuilt on the GPU in stream order (no host read-back)."""
        if lam.numel() != self.batch:
            raise ValueError("lambda needs one value per instance")
        self._check(lib().tmg_set_lambda(self._h, _ptr(lam), _stream()), "tmg_set_lambda")

    def set_active_set(self, on):
        """Later cycles of a batch on the running instances' tiles only
        (on by default; the results are bitwise the same either way)."""
        self._check(lib().tmg_set_active_set(self._h, int(bool(on))), "tmg_set_active_set")

    def set_dense_bottom(self, on):
        """The bottom level's visits (V or W) as one precomputed dense
        operator (on by default; the same cycle up to rounding); off: the
        bottom kernel's recursion at every visit."""
        self._check(lib().tmg_set_dense_bottom(self._h, int(bool(on)), _stream()),
                    "tmg_set_dense_bottom")

    def vcycle(self, f, u0, u):
        self._check(lib().tmg_vcycle(self._h, _ptr(f), _ptr(u0), _ptr(u), _stream()),
                    "tmg_vcycle")
        return u

    def adjoint_solve(self, g, u=None, z=None, rtol=1e-10, max_cycles=100):
        """Returns (z, dlambda[batch], du0[batch], cycles, relres, status)."""
        if z is None:
            z = torch.empty_like(g)
        dl = (ctypes.c_double * self.batch)()
        du = (ctypes.c_double * self.batch)()
        cyc = (ctypes.c_int * self.batch)()
        rr = (ctypes.c_double * self.batch)()
        rc = lib().tmg_adjoint_solve(self._h, _ptr(g), _ptr(u), _ptr(z), rtol, max_cycles, dl, du,
                                     cyc, rr, _stream())
        self._check(rc, "tmg_adjoint_solve")
        return z, list(dl), list(du), list(cyc), list(rr), rc

    # -- level-wise kernels ----------------------------------------------
    def level_info(self, j: int, level: int):
        n = ctypes.c_int64()
        a = ctypes.c_double()
        w = ctypes.c_double()
        rc = lib().tmg_level_info(self._h, j, level, ctypes.byref(n), ctypes.byref(a),
                                  ctypes.byref(w))
        self._check(rc, "tmg_level_info")
        return rc, n.value, a.value, w.value

    def level_size(self, level: int) -> int:
        return int(lib().tmg_level_size(self._h, level))

    def down(self, level, f, u_in=None, u_out=None, rc=None, nsweep=2, trans=False,
             fold_u0=None):
        r = lib().tmg_op_down(self._h, level, int(trans), nsweep, _ptr(f), _ptr(fold_u0),
                              _ptr(u_in), _ptr(u_out), _ptr(rc), _stream())
        self._check(r, "tmg_op_down")

    def up(self, level, f, u_in, e=None, u_out=None, nsweep=2, trans=False, fold_u0=None):
        r = lib().tmg_op_up(self._h, level, int(trans), nsweep, _ptr(f), _ptr(fold_u0),
                            _ptr(u_in), _ptr(e), _ptr(u_out), _stream())
        self._check(r, "tmg_op_up")

    def fused(self, f, u_in, e, u_out, rc, trans=False, fold_u0=None):
        r = lib().tmg_op_fused(self._h, int(trans), _ptr(f), _ptr(fold_u0), _ptr(u_in), _ptr(e),
                               _ptr(u_out), _ptr(rc), _stream())
        self._check(r, "tmg_op_fused")

    def fused2(self, f, u_in, f1, e2, u_out, rc, f2=None, trans=False, fold_u0=None):
        r = lib().tmg_op_fused2(self._h, int(trans), _ptr(f), _ptr(fold_u0), _ptr(u_in), _ptr(f1),
                                _ptr(e2), _ptr(u_out), _ptr(rc), _ptr(f2), _stream())
        self._check(r, "tmg_op_fused2")

    def down32(self, level, f, u_in=None, u_out=None, rc=None, nsweep=2, trans=False):
        """FP32 down leg (precision = 1 handles); float32 tensors."""
        r = lib().tmg_op_down32(self._h, level, int(trans), nsweep, _ptr32(f), _ptr32(u_in),
                                _ptr32(u_out), _ptr32(rc), _stream())
        self._check(r, "tmg_op_down32")

    def up32(self, level, f, u_in, e=None, u_out=None, nsweep=2, trans=False):
        """FP32 up leg (precision = 1 handles); float32 tensors."""
        r = lib().tmg_op_up32(self._h, level, int(trans), nsweep, _ptr32(f), _ptr32(u_in),
                              _ptr32(e), _ptr32(u_out), _stream())
        self._check(r, "tmg_op_up32")

    def mix(self, f, u_in, e, u_out, rc, trans=False, fold_u0=None):
        """Level-0 pass of an FP32-inner outer iteration: f, u_in, u_out float64,
        e and rc float32 (level 1's layout)."""
        r = lib().tmg_op_mix(self._h, int(trans), _ptr(f), _ptr(fold_u0), _ptr(u_in), _ptr32(e),
                             _ptr(u_out), _ptr32(rc), _stream())
        self._check(r, "tmg_op_mix")

    def coarse_solve(self, level, r, e, trans=False):
        rc = lib().tmg_op_coarse_solve(self._h, level, int(trans), _ptr(r), _ptr(e), _stream())
        self._check(rc, "tmg_op_coarse_solve")

    def residual_norm(self, f, u, fold_u0=None, trans=False):
        out = (ctypes.c_double * self.batch)()
        rc = lib().tmg_op_residual_norm(self._h, int(trans), _ptr(f), _ptr(fold_u0), _ptr(u),
                                        out, _stream())
        self._check(rc, "tmg_op_residual_norm")
        return list(out)


class HeatSolver:
    """The space-time heat equation u_t - u_xx = f on (0,1), u = 0 at both
    ends, nx interior points, N slabs on (0, T]: arrays [point][slab][k]
    (flat float64 device tensors); u0 has nx values."""

    def __init__(self, n_slabs, nx, T, **opts):
        self.N, self.nx, self.T = int(n_slabs), int(nx), float(T)
        self.opts = Options.make(**opts)
        self.P = self.opts.p + 1
        self.size = self.N * self.nx * self.P
        h = ctypes.c_void_p()
        rc = lib().tmg_heat_setup(ctypes.byref(h), self.N, self.nx, self.T,
                                  ctypes.byref(self.opts), _stream())
        if rc != TMG_OK:
            raise TmgError(rc, "tmg_heat_setup")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().tmg_heat_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, where):
        if rc < 0:
            raise TmgError(rc, where, lib().tmg_heat_last_hip_error(self._h))
        return rc

    def set_mode_solve(self, on):
        """The coarse levels by sine modes (on by default; the same cycle up
        to rounding); off: their legs."""
        self._check(lib().tmg_heat_set_mode_solve(self._h, int(bool(on))),
                    "tmg_heat_set_mode_solve")

    def vcycle(self, f, u0, u):
        self._check(lib().tmg_heat_vcycle(self._h, _ptr(f), _ptr(u0), _ptr(u), _stream()),
                    "tmg_heat_vcycle")
        return u

    def solve(self, f, u0, u=None, rtol=1e-10, max_cycles=100) -> SolveResult:
        if u is None:
            u = torch.empty_like(f)
        cyc = (ctypes.c_int * 1)()
        rr = (ctypes.c_double * 1)()
        rc = lib().tmg_heat_solve(self._h, _ptr(f), _ptr(u0), _ptr(u), rtol, max_cycles, cyc, rr,
                                  _stream())
        self._check(rc, "tmg_heat_solve")
        return SolveResult(u, list(cyc), list(rr), rc)
