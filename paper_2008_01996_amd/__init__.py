"""stfd: space-time Fast Diagonalization (Langer & Zank, arXiv 2008.01996) on MI355X.

The solver lives in the C library libstfd.so (include/stfd.h); this package
holds its sources (csrc/), the build script and the ctypes binding.
"""
from .stfd import (EINVAL, ENOCONV, ENOMEM, ENUMERIC, ESTATE, EHIP, OK, Batch, Problem, Space, StfdError,  # noqa: F401
                   assemble_time, lib, time_decompose, time_schur)
