"""MI355X-native low-rank Poisson solver (Cross-DEIM with leverage scores).

The solver lives in the HIP library liblrp.so (C-ABI declared in include/lrp.h); this
package holds its sources (csrc/), the in-tree build script and the ctypes binding.
"""
from .lrp import LRP_FP64, LRP_MIXED, LrpError, Solver, fortran, lib  # noqa: F401
