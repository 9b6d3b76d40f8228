"""MI355X (gfx950) IFEAST: FEAST contour integration with inexact block-GMRES solves.

A thin Python binding over the C ABI of ``libifeast.so`` (``include/ifeast.h``):
it marshals arguments only; every step of the solver runs in the library's
HIP kernels.  PyTorch is used for device buffers and streams in the
device-pointer entry points.  The package raises if the library has not been
built (``python -m paper_1706_00692_amd.build``); there is no CPU fallback.
"""

from ._binding import (
    IFeastError,
    Context,
    Matrix,
    Result,
    contour_struct,
    params_struct,
    problem_params,
    footprint,
    library_path,
    load_library,
    exported_symbols,
    PREC_FP64,
    PREC_MIXED,
    BASIS_AUTO,
    BASIS_SHARED,
    BASIS_PER_SHIFT,
    BASIS_MINRES,
    FLAG_INSIDE,
    FLAG_SPURIOUS,
    STATUS,
)

__all__ = [
    "IFeastError",
    "Context",
    "Matrix",
    "Result",
    "contour_struct",
    "params_struct",
    "problem_params",
    "footprint",
    "library_path",
    "load_library",
    "exported_symbols",
    "PREC_FP64",
    "PREC_MIXED",
    "BASIS_AUTO",
    "BASIS_SHARED",
    "BASIS_PER_SHIFT",
    "BASIS_MINRES",
    "FLAG_INSIDE",
    "FLAG_SPURIOUS",
    "STATUS",
]
