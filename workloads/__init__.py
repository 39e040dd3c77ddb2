"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This package holds no part of the multigrid method: it only draws
random numbers and forms DG load vectors (integrals of f against the Legendre
basis of each slab), which are the inputs of the solve."""
from .gen import *  # noqa: F401,F403
