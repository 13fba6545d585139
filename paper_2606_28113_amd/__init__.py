"""MI355X (gfx950) symmetric Gauss-Seidel projection method for the Landau-Lifshitz equation.

Thin Python binding of ``libsgspm.so`` (C ABI in ``include/sgspm.h``): argument
marshalling only.  Every step of the method runs in the library's HIP kernels;
PyTorch supplies device memory and the stream.  Importing this package fails
loudly when the library has not been built (``__graft_entry__.build()`` or
``python paper_2606_28113_amd/build.py``).
"""
import ctypes
import os

from .binding import (  # noqa: F401
    FP32, FP64, SCHEME_GS, SCHEME_SGS, SCHEME_SGS_FF, TERM_ALL, TERM_ANISO, TERM_EXCHANGE, TERM_STRAY, TERM_ZEEMAN,
    UNITS_REDUCED, UNITS_SI, Plan, SGSPMError, lib, lib_path, reduced_constants, validate,
)
from .autograd import SGSPMFunction, run_steps  # noqa: F401
