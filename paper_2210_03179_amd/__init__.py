"""MI355X-native Chebyshev-smoothed p-multigrid PCG for spectral-element Poisson.

Implements the solver path of Phillips & Fischer, "Optimal Chebyshev Smoothers
and One-sided V-cycles" (arXiv 2210.03179) as hand-written HIP kernels behind
the C ABI of include/semcheb.h (libsemcheb.so). This package is the thin Python
binding over that library.
"""
from ._lib import SemError, load, LIB_PATH  # noqa: F401
from .solver import SemSolver, FdSolver, BatchedSolver, SolveInfo, beta_table  # noqa: F401
