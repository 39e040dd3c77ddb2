"""Build the HIP library ``_lib/libtmg.so`` for gfx950 with hipcc.

Usage: ``python -m paper_1409_5254_amd.build`` (always recompiles).  Every
source compiles to its own object in parallel; one link makes the library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libtmg.so")
# (source, extra flags, object name); the bottom kernel and the generic
# kernels are compiled once per P.  Largest translation units first, so that they start first.
SOURCES = ([("tmg_bottom.hip", [f"-DTMG_BOTTOM_P={p}"], f"tmg_bottom_p{p}") for p in (6, 5, 4, 3, 2, 1)]
           + [("tmg_generic.hip", [f"-DTMG_GEN_P={p}"], f"tmg_generic_p{p}") for p in range(21, 0, -1)]
           + [(s, [], os.path.splitext(s)[0]) for s in
              ("tmg_leg64.hip", "tmg_leg32.hip", "tmg_span.hip", "tmg_mix.hip", "tmg_capi.cpp",
               "tmg_heat.hip", "tmg_heat_capi.cpp", "tmg_kernels.hip", "tmg_dense.hip", "tmg_tables.cpp")])
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
              shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags() -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # no packed-FP32 instructions (v_pk_*_f32) in any device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source for gfx950 into one shared library (always)."""
    os.makedirs(LIBDIR, exist_ok=True)
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    with tempfile.TemporaryDirectory(prefix="tmgbuild") as tmpd:
        def compile_one(item):
            src, extra, name = item
            obj = os.path.join(tmpd, name + ".o")
            cmd = [cc] + flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
            res = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, res
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, SOURCES))
        failed = False
        for src, _, res in results:
            if res.returncode != 0:
                sys.stderr.write(f"--- {src}\n{res.stdout}{res.stderr}")
                failed = True
            elif verbose and res.stderr.strip():
                sys.stderr.write(f"--- {src}\n{res.stderr}")
        if failed:
            raise RuntimeError("hipcc failed")
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc link failed")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
