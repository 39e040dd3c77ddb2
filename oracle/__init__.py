"""FP64 CPU oracle for the DG-in-time time-multigrid solve (Gander & Neumueller).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute anything
in this package.  It shares no code with the HIP library
(``paper_1409_5254_amd``) and never imports it; the HIP library never imports
this package.

* ``oracle.core``     -- ctypes wrapper around ``tmg_oracle.c`` (plain C, FP64,
  built with ``-O2 -ffp-contract=off``): slab matrices, direct solve, Jacobi
  sweeps, residual, transfers, reference V/W cycle and solve, transposed
  (adjoint) system, gradients, and the mixed-precision reference.
* ``oracle.analysis`` -- NumPy tools taken from the paper's analysis: the
  printed Pade stability functions, left Radau nodes, dense assembly of the
  global system, and the two-grid Fourier symbol of Theorem chap4_theorem4.
"""
