"""MI355X (gfx950) time-multigrid solver for DG-in-time discretisations of
u' + lambda u = f (Gander & Neumueller, arXiv:1409.5254).

The solve runs in the HIP library ``_lib/libtmg.so`` (C ABI in
``include/tmg.h``); this package holds its sources (``csrc/``), the build
step (``build``), the ctypes binding (``binding``) and the autograd wrapper
(``autograd``).  Importing the package does not load torch or the library.
"""

__all__ = ["binding", "autograd", "build"]
