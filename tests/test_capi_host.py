"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/tmg.h declares, and rejects invalid arguments before any
device work (status codes of the header)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1409_5254_amd import binding
    if not os.path.exists(binding._LIB_PATH):
        pytest.skip("HIP library not built")
    return binding


def test_header_symbols_exported():
    b = _lib()
    hdr = open(os.path.join(ROOT, "include", "tmg.h")).read()
    declared = set(re.findall(r"\b(tmg_[a-z_0-9]+)\s*\(", hdr))
    L = b.lib()
    missing = [s for s in declared if not hasattr(L, s)]
    assert not missing
    assert declared == set(b.SYMBOLS)


def test_error_strings():
    b = _lib()
    for code in [0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10]:
        assert b.error_string(code)
    assert "unknown" in b.error_string(12345)


def _setup(b, n, T, lam, **kw):
    o = b.Options.make(**kw)
    h = ctypes.c_void_p()
    k = len(n)
    return b.lib().tmg_setup(ctypes.byref(h), k, (ctypes.c_int64 * k)(*n),
                             (ctypes.c_double * k)(*T), (ctypes.c_double * k)(*lam),
                             ctypes.byref(o), None)


@pytest.mark.parametrize("n,T,lam,kw,code", [
    ([1000], [1.0], [1.0], {}, -2),                       # not n_coarse * 2^k
    ([1024], [1.0], [1.0], dict(n_coarse=3), -2),
    ([1024], [0.0], [1.0], {}, -4),                       # T <= 0
    ([1024], [1.0], [-1.0], {}, -4),                      # lambda <= 0
    ([1024], [1.0], [float("nan")], {}, -4),
    ([1024], [1.0], [1.0], dict(p=21), -1),               # degree not built (0..20)
    ([1024], [1.0], [1.0], dict(p=30), -1),
    ([1024], [1.0], [1.0], dict(periodic=2), -1),
    ([1024], [1.0], [1.0], dict(p=10, precision=1), -9),  # FP32-inner: tuned degrees only
    ([1024], [1.0], [1.0], dict(periodic=1, precision=1), -9),
    ([1024], [1.0], [1.0], dict(p=-1), -1),
    ([1024], [1.0], [1.0], dict(gamma=3), -1),
    ([1024], [1.0], [1.0], dict(nu1=9), -1),
    ([1024], [1.0], [1.0], dict(omega_mode=1, omega=1.5), -3),
    ([1024], [1.0], [1.0], dict(omega_mode=1, omega=0.0), -3),
    ([1024], [1.0], [1.0], dict(precision=7), -9),
    ([1024, 96], [1.0, 1.0], [1.0, 1.0], {}, -2),
])
def test_setup_rejects(n, T, lam, kw, code):
    b = _lib()
    assert _setup(b, n, T, lam, **kw) == code


def test_null_arguments():
    b = _lib()
    L = b.lib()
    assert L.tmg_setup(None, 1, None, None, None, None, None) == -1
    assert L.tmg_solve(None, None, None, None, 1e-10, 10, None, None, None) == -1
    assert L.tmg_vcycle(None, None, None, None, None) == -1
    assert L.tmg_destroy(None) == -1
    assert L.tmg_level_size(None, 0) == -1
    assert L.tmg_set_active_set(None, 1) == -1
    assert L.tmg_set_dense_bottom(None, 1, None) == -1
    assert L.tmg_heat_set_mode_solve(None, 1) == -1
    o = b.Options.make(p=1)
    assert L.tmg_solve_noalloc(1024, 1.0, 1.0, None, None, None, None, 1e-10, 10, None, None,
                               None) == -1
    assert L.tmg_solve_noalloc(1024, 1.0, 1.0, ctypes.byref(o), None, None, None, 1e-10, 10,
                               None, None, None) == -1


@pytest.mark.parametrize("n,p,kw,code", [
    (1 << 21, 1, {}, -2),            # N * P = 2^22, above the no-alloc limit of 2^21
    (1 << 19, 3, {}, -2),
    (1000, 1, {}, -2),               # not n_coarse * 2^k
    (1024, 1, dict(gamma=3), -1),
    (1024, 1, dict(omega_mode=1, omega=2.0), -3),
])
def test_noalloc_rejects_before_device_work(n, p, kw, code):
    """tmg_solve_noalloc checks its arguments and the size limit on the host
    before it touches a device (the pointers are never dereferenced)."""
    b = _lib()
    o = b.Options.make(p=p, **kw)
    fake = ctypes.c_void_p(256)
    if (n, p) == (1 << 19, 3):
        n = (1 << 19) + (1 << 18)   # 3 * 2^18 slabs: N * P above 2^21, n_coarse 3 * 2^k
        o.n_coarse = 3
    assert b.lib().tmg_solve_noalloc(n, 1.0, 1.0, ctypes.byref(o), fake, fake, fake, 1e-10, 10,
                                     None, None, None) == code


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU only: --gpus N > 1 exits with a message
    (before anything touches a GPU)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n,nx,T,kw,code", [
    (1024, 0, 1.0, {}, -1),
    (1024, 5000, 1.0, {}, -1),            # above TMG_HEAT_MAX_POINTS
    (1024, 15, 1.0, dict(p=6), -1),       # the heat solver takes the tuned degrees
    (1024, 15, 1.0, dict(precision=1), -9),
    (1024, 15, 1.0, dict(periodic=1), -9),
    (1000, 15, 1.0, {}, -2),              # not n_coarse * 2^k
    (2, 15, 1.0, {}, -2),                 # one level only
    (1024, 15, 0.0, {}, -4),
    (1024, 15, 1.0, dict(omega_mode=1, omega=1.5), -3),
])
def test_heat_setup_rejects(n, nx, T, kw, code):
    """tmg_heat_setup checks its arguments before any device work."""
    b = _lib()
    o = b.Options.make(**kw)
    h = ctypes.c_void_p()
    assert b.lib().tmg_heat_setup(ctypes.byref(h), n, nx, T, ctypes.byref(o), None) == code
