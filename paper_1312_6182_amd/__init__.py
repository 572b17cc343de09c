"""GP-SPCA (generalized power method for sparse PCA) on MI355X / gfx950.

The compute path is the HIP library libgpspca.so (C ABI in include/gpspca.h);
this package is a thin binding over it.  PyTorch is used only for device
memory and streams.
"""
from ._lib import (  # noqa: F401
    SL1, SL0, BL1, BL0, BL1X, F32, BF16, F8E4M3,
    OK, MAXITER, DEGENERATE, EINVAL, EDTYPE, ENOMEM, EDEVICE, ENONFINITE, MAX_M,
    NOALLOC_SCRATCH_BYTES,
    GpspcaError, load, last_error, LIB_PATH, SIGNATURES,
)


def __getattr__(name):
    # torch-facing helpers are imported lazily so that loading the C library
    # (e.g. for symbol checks) does not require a GPU.
    if name in ("solve", "step", "column_norms", "workspace_bytes", "matrix", "column_major",
                "profile_enable", "profile_read", "SolveResult", "StepResult", "solve_path",
                "solve_multistart", "solve_deflated", "solve_noalloc",
                "PathResult", "quantize", "refine", "refine_path", "autotune", "autotune_clear"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
