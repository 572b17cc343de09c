"""FP64 CPU oracle of the GP-SPCA power iteration -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it.  The arithmetic lives in ``gpspca_oracle.c`` (plain double-precision
loops, one function per step of the method); this module only marshals NumPy
arrays through ctypes and builds the C library with gcc when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

SL1, SL0, BL1, BL0 = 0, 1, 2, 3
# block L1 read from its original form (objective sum_j ||s_j||, direction
# mu_j A s_j / ||s_j||); see orc_bl1x_direction
BL1X = 4
OK, MAXITER, DEGENERATE = 0, 1, 2
EINVAL, ENOMEM, ENONFINITE = -1, -3, -5

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpspca_oracle.c")
# GPSPCA_ORACLE_LIB names a separately built copy (the sanitizer test's
# instrumented build); it is used as given and never rebuilt here.
_LIB_ENV = os.environ.get("GPSPCA_ORACLE_LIB")
_LIB = _LIB_ENV or os.path.join(_HERE, "libgpspca_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, OpenMP)."""
    if _LIB_ENV:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
            P = ctypes.c_void_p
            L.orc_column_norms.argtypes = [P, i64, i64, i64, P]
            L.orc_top_m.argtypes = [P, i64, i32, P]
            L.orc_polar.argtypes = [P, i64, i32, P, P, P]
            L.orc_pass.argtypes = [P, i64, i64, i64, i32, i32, d, P, P, P, P, P, P, P, P]
            L.orc_retract.argtypes = [i64, i32, P, P, P, P, P]
            L.orc_bl1x_direction.argtypes = [i64, i32, P, P]
            L.orc_bl1x_direction.restype = d
            L.orc_project.argtypes = [i64, i32, P, P]
            L.orc_init.argtypes = [P, i64, i64, i64, i32, P, P]
            L.orc_solve.argtypes = [P, i64, i64, i64, i32, i32, d, P, P, P, d, i32, P, P, P, P, P]
            L.orc_encode.argtypes = [P, i64, i32, P]
            L.orc_decode.argtypes = [P, i64, i32, P]
            L.orc_quantize.argtypes = [P, i64, i64, i64, i32, P, i64, P]
            L.orc_dequantize.argtypes = [P, i64, i64, i64, i32, P, P]
            L.orc_set_num_threads.argtypes = [i32]
            for name in ("orc_column_norms", "orc_top_m", "orc_polar", "orc_pass", "orc_retract",
                         "orc_project", "orc_init", "orc_solve", "orc_num_threads", "orc_encode",
                         "orc_decode", "orc_quantize", "orc_dequantize"):
                getattr(L, name).restype = i32
            L.orc_set_num_threads.restype = None
            _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} returned {code}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _matrix(A):
    """Column-major FP64 view of A: returns (array, p, n, lda)."""
    A = np.asarray(A)
    if A.ndim == 1:
        A = A.reshape(-1, 1)
    A = np.asfortranarray(A, dtype=np.float64)
    p, n = A.shape
    return A, p, n, p


def set_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def column_norms(A):
    A, p, n, lda = _matrix(A)
    c = np.empty(n)
    rc = lib().orc_column_norms(_ptr(A), p, n, lda, _ptr(c))
    if rc:
        raise OracleError(rc, "orc_column_norms")
    return c


def top_m(c, m: int):
    c = np.ascontiguousarray(c, dtype=np.float64)
    idx = np.empty(m, dtype=np.int64)
    rc = lib().orc_top_m(_ptr(c), c.size, m, _ptr(idx))
    if rc:
        raise OracleError(rc, "orc_top_m")
    return idx


def polar(G):
    """Polar factor of G by one-sided Jacobi; returns (X, singular values, rank_deficient)."""
    G = np.asfortranarray(G, dtype=np.float64)
    p, m = G.shape
    X = np.empty((p, m), order="F")
    sv = np.empty(m)
    rd = ctypes.c_int(0)
    rc = lib().orc_polar(_ptr(G), p, m, _ptr(X), _ptr(sv), ctypes.byref(rd))
    if rc:
        raise OracleError(rc, "orc_polar")
    return X, sv, bool(rd.value)


def _mask(mask, n, m):
    if mask is None:
        return None
    mk = np.asfortranarray(np.asarray(mask, dtype=np.uint8).reshape(n, m))
    return mk


def step(A, form: int, X, gamma: float, mu=None, mask=None):
    """One pass at X.  Returns dict(Y, S, G, f, nnz, F).  mask (n x m bool, or
    None) forces s_ij = 0 where it is False (pass on a frozen support)."""
    A, p, n, lda = _matrix(A)
    X = np.asfortranarray(np.asarray(X, dtype=np.float64).reshape(p, -1))
    m = X.shape[1]
    muv = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
    Y = np.empty((n, m), order="F")
    S = np.empty((n, m), order="F")
    G = np.empty((p, m), order="F")
    f = np.empty(m)
    nnz = np.empty(m, dtype=np.int64)
    mk = _mask(mask, n, m)
    rc = lib().orc_pass(_ptr(A), p, n, lda, form, m, float(gamma), _ptr(muv), _ptr(X), _ptr(mk),
                        _ptr(Y), _ptr(S), _ptr(G), _ptr(f), _ptr(nnz))
    if rc:
        raise OracleError(rc, "orc_pass")
    if form == BL1X:
        # objective sum_j ||s_j|| and direction mu_j A s_j / ||s_j||
        F = float(lib().orc_bl1x_direction(p, m, _ptr(f), _ptr(G)))
        return dict(Y=Y, S=S, G=G, f=f, nnz=nnz, F=F)
    return dict(Y=Y, S=S, G=G, f=f, nnz=nnz, F=float(f.sum()))


def retract(G, nnz, Xk):
    G = np.asfortranarray(G, dtype=np.float64)
    p, m = G.shape
    nnz = np.ascontiguousarray(nnz, dtype=np.int64)
    Xk = np.asfortranarray(Xk, dtype=np.float64)
    Xn = np.empty((p, m), order="F")
    deg = ctypes.c_int(0)
    rc = lib().orc_retract(p, m, _ptr(G), _ptr(nnz), _ptr(Xk), _ptr(Xn), ctypes.byref(deg))
    if rc:
        raise OracleError(rc, "orc_retract")
    return Xn, bool(deg.value)


def project(X0):
    X0 = np.asfortranarray(X0, dtype=np.float64)
    if X0.ndim == 1:
        X0 = X0.reshape(-1, 1)
    p, m = X0.shape
    X = np.empty((p, m), order="F")
    rc = lib().orc_project(p, m, _ptr(X0), _ptr(X))
    if rc:
        raise OracleError(rc, "orc_project")
    return X


def init(A, m: int):
    """Default start: polar factor (or normalization) of the m largest-norm columns."""
    A, p, n, lda = _matrix(A)
    X = np.empty((p, m), order="F")
    idx = np.empty(m, dtype=np.int64)
    rc = lib().orc_init(_ptr(A), p, n, lda, m, _ptr(X), _ptr(idx))
    if rc:
        raise OracleError(rc, "orc_init")
    return X, idx


def solve(A, form: int, m: int, gamma: float, mu=None, X0=None, tol: float = 1e-4,
          max_iter: int = 1000, mask=None):
    """Full solve.  Returns dict(X, Z, support, trace, n_iter, status).  With a
    mask (n x m bool), every pass is restricted to that frozen support."""
    A, p, n, lda = _matrix(A)
    muv = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
    X0v = None if X0 is None else np.asfortranarray(np.asarray(X0, dtype=np.float64).reshape(p, -1))
    X = np.empty((p, m), order="F")
    Z = np.empty((n, m), order="F")
    sup = np.empty((n, m), dtype=np.uint8, order="F")
    trace = np.zeros(max_iter)
    nit = ctypes.c_int(0)
    mk = _mask(mask, n, m)
    rc = lib().orc_solve(_ptr(A), p, n, lda, form, m, float(gamma), _ptr(muv), _ptr(X0v), _ptr(mk),
                         float(tol), int(max_iter), _ptr(X), _ptr(Z), _ptr(sup), _ptr(trace),
                         ctypes.byref(nit))
    if rc < 0:
        raise OracleError(rc, "orc_solve")
    k = nit.value
    return dict(X=X, Z=Z, support=sup.astype(bool), trace=trace[:k].copy(), n_iter=k, status=rc)


def solve_deflated(A, form: int, m: int, gamma: float, tol: float = 1e-4, max_iter: int = 1000):
    """m single-unit components by projection deflation (the paper times its
    single-unit formulations with several components, Section 4.1, without
    stating how they are obtained; this is the reading): component k is the
    single-unit solve (form SL1 or SL0) on A_k = (I - X_{<k} X_{<k}^T) A from
    the default start of A_k, its normalized column of largest norm.  Each
    deflation is applied explicitly in FP64.  Returns dict(X, Z, support,
    traces, n_iter, status) with one column / entry per component."""
    A = np.asarray(A, dtype=np.float64)
    p, n = A.shape
    X = np.zeros((p, m), order="F")
    Z = np.zeros((n, m), order="F")
    sup = np.zeros((n, m), dtype=bool)
    traces, n_iter, status = [], [], []
    Ak = np.array(A, order="F")
    for k in range(m):
        if k > 0:
            q = X[:, k - 1:k]
            Ak = np.asfortranarray(Ak - q @ (q.T @ Ak))
        r = solve(Ak, form, 1, gamma, tol=tol, max_iter=max_iter)
        X[:, k] = r["X"][:, 0]
        Z[:, k] = r["Z"][:, 0]
        sup[:, k] = r["support"][:, 0]
        traces.append(r["trace"])
        n_iter.append(r["n_iter"])
        status.append(r["status"])
    return dict(X=X, Z=Z, support=sup, traces=traces, n_iter=n_iter, status=status)


# ---------------------------------------------------------------- storage
BF16, E4M3 = 1, 2


def encode(v, to: int) -> np.ndarray:
    """Element-wise bfloat16 (to=1, uint16 codes) or e4m3fn (to=2, uint8 codes)
    rounding of FP32 values, no scaling."""
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float32).ravel())
    out = np.empty(v.size, dtype=np.uint16 if to == BF16 else np.uint8)
    rc = lib().orc_encode(_ptr(v), v.size, int(to), _ptr(out))
    if rc:
        raise OracleError(rc, "orc_encode")
    return out


def decode(c, to: int) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(c, dtype=np.uint16 if to == BF16 else np.uint8).ravel())
    out = np.empty(c.size)
    rc = lib().orc_decode(_ptr(c), c.size, int(to), _ptr(out))
    if rc:
        raise OracleError(rc, "orc_decode")
    return out


def quantize(A32, to: int, ldq: int | None = None):
    """Codes (ldq x n column-major array, rows >= p unspecified) and per-column
    scales of the FP32 matrix A32 (p x n)."""
    A32 = np.asfortranarray(np.asarray(A32, dtype=np.float32))
    p, n = A32.shape
    ldq = p if ldq is None else int(ldq)
    codes = np.zeros((ldq, n), dtype=np.uint16 if to == BF16 else np.uint8, order="F")
    scale = np.empty(n, dtype=np.float32)
    rc = lib().orc_quantize(_ptr(A32), p, n, p, int(to), _ptr(codes), ldq, _ptr(scale))
    if rc:
        raise OracleError(rc, "orc_quantize")
    return codes, scale


def dequantize(codes, to: int, scale, p: int) -> np.ndarray:
    """FP64 (p x n) matrix of code_value * scale_i."""
    codes = np.asfortranarray(codes)
    ldq, n = codes.shape
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float32)
    out = np.empty((p, n), order="F")
    rc = lib().orc_dequantize(_ptr(codes), p, n, ldq, int(to), _ptr(sc), _ptr(out))
    if rc:
        raise OracleError(rc, "orc_dequantize")
    return out
