"""rIGA shift-and-invert eigensolver for the MI355X (gfx950).

The solver lives in libriga.so (HIP kernels + host runtime behind the C ABI
of include/riga.h); ``riga`` is its ctypes binding.
"""
from . import riga  # noqa: F401
from .riga import (RIGA_FP64, RIGA_MIXED, RIGA_MAT_A, RIGA_MAT_K, RIGA_MAT_M,  # noqa: F401
                   EigSum, Problem, RigaError, analyze, assemble, eigs)
