"""ctypes binding of libgpspca.so (the gfx950 C ABI declared in include/gpspca.h).

Marshalling only: every step of the method runs in the HIP library.  Loading
fails loudly when the shared library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpspca.so")

SL1, SL0, BL1, BL0 = 0, 1, 2, 3
BL1X = 4  # block L1 from its original form (gpspca_solve only)
F32, BF16, F8E4M3 = 0, 1, 2
OK, MAXITER, DEGENERATE = 0, 1, 2
EINVAL, EDTYPE, ENOMEM, EDEVICE, ENONFINITE = -1, -2, -3, -4, -5
MAX_M = 64
NOALLOC_SCRATCH_BYTES = 64 << 20


class Matrix(ctypes.Structure):
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("p", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("col_scale", ctypes.c_void_p),
    ]


class GpspcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpspca error {code}: {msg}")
        self.code = code


_lock = threading.Lock()
_lib = None

# (name, restype, argtypes) of every exported entry point
_P, _I, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_MP = ctypes.POINTER(Matrix)
SIGNATURES = {
    "gpspca_workspace_bytes": (_SZ, [_MP, _I, _I, _I]),
    "gpspca_solve": (_I, [_MP, _I, _I, _D, _P, _P, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P]),
    "gpspca_solve_noalloc": (_I, [_MP, _I, _I, _D, _P, _P, _D, _I, _P, _P, _P, _P, _P, _P]),
    "gpspca_step": (_I, [_MP, _I, _I, _D, _P, _P, _P, _SZ, _P, _P, _P, _P, _P]),
    "gpspca_column_norms": (_I, [_MP, _P, _P]),
    "gpspca_path_workspace_bytes": (_SZ, [_MP, _I, _I]),
    "gpspca_solve_path": (_I, [_MP, _I, _I, _P, _P, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P, _P]),
    "gpspca_solve_multistart": (_I, [_MP, _I, _I, _D, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P,
                                     _P]),
    "gpspca_deflated_workspace_bytes": (_SZ, [_MP, _I, _I]),
    "gpspca_solve_deflated": (_I, [_MP, _I, _I, _D, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P,
                                   _P]),
    "gpspca_refine": (_I, [_MP, _I, _I, _D, _P, _P, _P, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P]),
    "gpspca_refine_path": (_I, [_MP, _I, _I, _P, _P, _P, _D, _I, _P, _SZ, _P, _P, _P, _P, _P, _P,
                                _P]),
    "gpspca_quantize": (_I, [_MP, _I, _P, _I64, _P, _P]),
    "gpspca_autotune": (_I, [_MP, _I, _I, _D, _P, _I, _P, _SZ, _P, _P, _P, ctypes.c_char_p, _SZ]),
    "gpspca_autotune_clear": (_I, []),
    "gpspca_last_error": (ctypes.c_char_p, []),
    "gpspca_version": (ctypes.c_char_p, []),
    "gpspca_profile_enable": (_I, [_I]),
    "gpspca_profile_read": (_I, [_P, _P, ctypes.c_char_p, _SZ]),
}


def load():
    """Load libgpspca.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_1312_6182_amd.build` (or __graft_entry__.build())")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def last_error() -> str:
    return load().gpspca_last_error().decode()


def check(rc: int, what: str) -> int:
    if rc < 0:
        raise GpspcaError(rc, f"{what}: {last_error()}")
    return rc
