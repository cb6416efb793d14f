"""MI355X (gfx950) solver for generalized DWD by the inexact sGS-ADMM.

The solver is the HIP library libdwd.so behind the C ABI in include/dwd.h;
``paper_2305_12019_amd.dwd`` is its ctypes binding.
"""
from . import dwd  # noqa: F401  (raises ImportError if libdwd.so is not built)
from .dwd import Problem, solve, params, footprint, DwdError  # noqa: F401
