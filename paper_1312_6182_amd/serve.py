"""Torch/NumPy-facing binding of the GP-SPCA solve server (gpspca_server_* in
include/gpspca.h): continuous batching of independent solves on one GPU.

PyTorch only provides the device arena; admission, residency, uploads and the
solves themselves run in libgpspca.so.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


class _Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("n_iter", ctypes.c_int), ("m", ctypes.c_int),
        ("uploaded", ctypes.c_int), ("p", ctypes.c_int64), ("n", ctypes.c_int64),
        ("X", ctypes.POINTER(ctypes.c_float)), ("Z", ctypes.POINTER(ctypes.c_float)),
        ("support", ctypes.POINTER(ctypes.c_uint32)),
        ("obj_trace", ctypes.POINTER(ctypes.c_double)),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("col_n_iter", ctypes.POINTER(ctypes.c_int)), ("col_status", ctypes.POINTER(ctypes.c_int)),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("waiting", "running", "completed", "uploads", "evictions")] + \
               [(k, ctypes.c_size_t) for k in ("resident_bytes", "free_bytes", "arena_bytes")]


_P, _I, _I64, _U64, _D, _SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                               ctypes.c_double, ctypes.c_size_t)
SIGNATURES = {
    "gpspca_server_create": (_I, [_P, _SZ, _I, ctypes.POINTER(_P)]),
    "gpspca_server_register": (_I, [_P, _P, _I64, _I64, _I64, _I, ctypes.POINTER(_U64)]),
    "gpspca_server_unregister": (_I, [_P, _U64]),
    "gpspca_server_submit": (_I, [_P, _U64, _I, _I, _D, _P, _D, _I, ctypes.POINTER(_U64)]),
    "gpspca_server_poll": (_I, [_P, _U64, ctypes.POINTER(_Result)]),
    "gpspca_server_wait": (_I, [_P, _U64, ctypes.POINTER(_Result)]),
    "gpspca_server_release": (_I, [_P, _U64]),
    "gpspca_server_stats": (_I, [_P, ctypes.POINTER(_Stats)]),
    "gpspca_server_destroy": (_I, [_P]),
}


def _lib():
    lib = L.load()
    if not getattr(lib, "_serve_sigs", False):
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._serve_sigs = True
    return lib


@dataclass
class ServeResult:
    X: np.ndarray            # (p, m)
    Z: np.ndarray            # (n, m)
    support: np.ndarray      # (m, ceil(n/32)) uint32 words
    trace: list              # multi-start: one list per problem
    n_iter: int
    status: int
    t_submit: float          # seconds on the server's clock
    t_admit: float
    t_done: float
    uploaded: bool
    col_n_iter: Optional[list] = None   # multi-start: passes and status per problem
    col_status: Optional[list] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit

    def support_mask(self) -> np.ndarray:
        m, nw = self.support.shape
        bits = (self.support[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1
        return bits.reshape(m, nw * 32)[:, :self.Z.shape[0]].T.astype(bool)


class Server:
    """A solve server over a device arena of `arena_bytes` with `slots`
    concurrent solves."""

    def __init__(self, arena_bytes: int, slots: int = 4):
        self._lib = _lib()
        buf = torch.empty(arena_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-buf.data_ptr()) % 256
        self._arena = buf[off:off + arena_bytes]
        self._h = _P()
        L.check(self._lib.gpspca_server_create(self._arena.data_ptr(), arena_bytes, slots,
                                               ctypes.byref(self._h)), "gpspca_server_create")
        self._host = {}

    def register(self, A: np.ndarray, store: str = "f32") -> int:
        """Register a host FP32 matrix (p, n); it is kept referenced (and must not
        be modified) until unregister."""
        A = np.asfortranarray(A, dtype=np.float32)
        p, n = A.shape
        mid = _U64()
        dt = {"f32": L.F32, "bf16": L.BF16}[store]
        L.check(self._lib.gpspca_server_register(self._h, A.ctypes.data, p, n, p, dt,
                                                 ctypes.byref(mid)), "gpspca_server_register")
        self._host[mid.value] = A
        return mid.value

    def unregister(self, mid: int) -> None:
        L.check(self._lib.gpspca_server_unregister(self._h, mid), "gpspca_server_unregister")
        self._host.pop(mid, None)

    def submit(self, mid: int, form: int, m: int, gamma: float,
               mu: Optional[Sequence[float]] = None, tol: float = 1e-4,
               max_iter: int = 1000) -> int:
        rid = _U64()
        mu_arr = None if mu is None else (ctypes.c_double * m)(*[float(v) for v in mu])
        L.check(self._lib.gpspca_server_submit(self._h, mid, form, m, float(gamma), mu_arr,
                                               float(tol), int(max_iter), ctypes.byref(rid)),
                "gpspca_server_submit")
        return rid.value

    @staticmethod
    def _convert(r: _Result) -> ServeResult:
        p, n, m, k = r.p, r.n, r.m, r.n_iter
        nw = (n + 31) // 32

        def arr(ptr, count, dtype):
            if not ptr or count == 0:
                return np.zeros(count, dtype=dtype)
            return np.ctypeslib.as_array(ptr, shape=(count,)).copy()

        X = arr(r.X, p * m, np.float32).reshape(m, p).T
        Z = arr(r.Z, n * m, np.float32).reshape(m, n).T
        sup = arr(r.support, nw * m, np.uint32).reshape(m, nw)
        cn = cs = None
        if r.col_n_iter:
            cn = [int(v) for v in arr(r.col_n_iter, m, np.int32)]
            cs = [int(v) for v in arr(r.col_status, m, np.int32)]
            flat = arr(r.obj_trace, m * k, np.float64)
            tr = [list(flat[j * k:j * k + cn[j]]) for j in range(m)]
        else:
            tr = list(arr(r.obj_trace, k, np.float64))
        return ServeResult(X=X, Z=Z, support=sup, trace=tr, n_iter=k, status=r.status,
                           t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done,
                           uploaded=bool(r.uploaded), col_n_iter=cn, col_status=cs)

    def poll(self, rid: int) -> Optional[ServeResult]:
        r = _Result()
        rc = self._lib.gpspca_server_poll(self._h, rid, ctypes.byref(r))
        if rc == 1:
            return None
        L.check(rc, "gpspca_server_poll")
        if r.status < 0:
            raise L.GpspcaError(r.status, L.last_error())
        return self._convert(r)

    def wait(self, rid: int, release: bool = True) -> ServeResult:
        r = _Result()
        L.check(self._lib.gpspca_server_wait(self._h, rid, ctypes.byref(r)), "gpspca_server_wait")
        if r.status < 0:
            msg = L.last_error()
            if release:
                self.release(rid)
            raise L.GpspcaError(r.status, msg)
        out = self._convert(r)
        if release:
            self.release(rid)
        return out

    def release(self, rid: int) -> None:
        L.check(self._lib.gpspca_server_release(self._h, rid), "gpspca_server_release")

    def stats(self) -> dict:
        s = _Stats()
        L.check(self._lib.gpspca_server_stats(self._h, ctypes.byref(s)), "gpspca_server_stats")
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def close(self) -> None:
        if self._h:
            L.check(self._lib.gpspca_server_destroy(self._h), "gpspca_server_destroy")
            self._h = _P()
            self._host.clear()
            self._arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
