"""Torch-facing wrappers of the GP-SPCA C ABI.

PyTorch provides device memory and the stream; every computation runs in
libgpspca.so.  A data matrix is a CUDA/HIP tensor ``A`` of shape (p, n) whose
columns are contiguous (``A.stride(0) == 1``, ``A.stride(1) = lda >= p``), e.g.
``At.t()`` for a contiguous (n, p) tensor ``At``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib as L

_DT = {torch.float32: L.F32, torch.bfloat16: L.BF16, torch.float8_e4m3fn: L.F8E4M3}


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def matrix(A: torch.Tensor, col_scale: Optional[torch.Tensor] = None) -> L.Matrix:
    """Describe a column-major device matrix (shape (p, n), stride (1, lda))."""
    if A.dim() != 2:
        raise ValueError("A must be 2-D (p, n)")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dtype not in _DT:
        raise ValueError(f"unsupported dtype {A.dtype}")
    p, n = A.shape
    if n > 1 and A.stride(0) != 1:
        raise ValueError("columns of A must be contiguous (stride(0) == 1)")
    lda = A.stride(1) if n > 1 else max(p, 1)
    if p > 1 and A.stride(0) != 1:
        raise ValueError("columns of A must be contiguous (stride(0) == 1)")
    M = L.Matrix()
    M.data = A.data_ptr()
    M.p, M.n, M.lda = p, n, lda
    M.dtype = _DT[A.dtype]
    M.col_scale = None if col_scale is None else col_scale.data_ptr()
    return M


def column_major(A_rows_are_columns: torch.Tensor) -> torch.Tensor:
    """View a contiguous (n, p) tensor (row i = column a_i) as the (p, n) matrix A."""
    return A_rows_are_columns.t()


def _mu_array(mu: Optional[Sequence[float]], m: int):
    if mu is None:
        return None
    arr = (ctypes.c_double * m)(*[float(v) for v in mu])
    if len(mu) != m:
        raise ValueError("mu must have m entries")
    return arr


def workspace_bytes(A: torch.Tensor, form: int, m: int, max_iter: int,
                    col_scale: Optional[torch.Tensor] = None) -> int:
    M = matrix(A, col_scale)
    nb = L.load().gpspca_workspace_bytes(ctypes.byref(M), form, m, max_iter)
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    return int(nb)


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


@dataclass
class SolveResult:
    X: torch.Tensor          # (p, m) column-major view
    Z: torch.Tensor          # (n, m) column-major view, unit-norm columns or 0
    support: torch.Tensor    # (m, ceil(n/32)) int32 bit words
    trace: list              # objective F_0 .. F_{n_iter-1}
    n_iter: int
    status: int

    def support_mask(self) -> torch.Tensor:
        """Boolean (n, m) support decoded from the bit words."""
        m, nw = self.support.shape
        n = self.Z.shape[0]
        bits = torch.arange(32, device=self.support.device, dtype=torch.int32)
        words = self.support.to(torch.int64) & 0xFFFFFFFF
        mask = ((words[:, :, None] >> bits[None, None, :]) & 1).bool()
        return mask.reshape(m, nw * 32)[:, :n].t()


def solve(A: torch.Tensor, form: int, m: int = 1, gamma: float = 0.0,
          mu: Optional[Sequence[float]] = None, X0: Optional[torch.Tensor] = None,
          tol: float = 1e-4, max_iter: int = 1000, col_scale: Optional[torch.Tensor] = None,
          stream: Optional[torch.cuda.Stream] = None,
          workspace: Optional[torch.Tensor] = None) -> SolveResult:
    """Run the GP-SPCA power iteration (gpspca_solve) on device tensor A (p, n)."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    dev = A.device
    nb = workspace_bytes(A, form, m, max_iter, col_scale)
    ws = workspace if workspace is not None and workspace.numel() >= nb else _workspace(nb, dev)
    Xt = torch.empty((m, p), dtype=torch.float32, device=dev)
    Zt = torch.empty((m, n), dtype=torch.float32, device=dev)
    nw = (n + 31) // 32
    sup = torch.empty((m, nw), dtype=torch.int32, device=dev)
    trace = (ctypes.c_double * max_iter)()
    nit = ctypes.c_int(0)
    x0p = None
    if X0 is not None:
        X0c = X0.t().contiguous() if X0.dim() == 2 else X0.reshape(1, -1).contiguous()
        if X0c.shape != (m, p) or X0c.dtype != torch.float32:
            raise ValueError("X0 must be a float32 (p, m) tensor")
        x0p = X0c.data_ptr()
    rc = lib.gpspca_solve(ctypes.byref(M), form, m, float(gamma), _mu_array(mu, m), x0p,
                          float(tol), int(max_iter), ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                          Xt.data_ptr(), Zt.data_ptr(), sup.data_ptr(), trace, ctypes.byref(nit))
    L.check(rc, "gpspca_solve")
    k = nit.value
    return SolveResult(X=Xt.t(), Z=Zt.t(), support=sup, trace=list(trace[:k]), n_iter=k,
                       status=rc)


def solve_noalloc(A: torch.Tensor, form: int, m: int = 1, gamma: float = 0.0,
                  mu: Optional[Sequence[float]] = None, X0: Optional[torch.Tensor] = None,
                  tol: float = 1e-4, max_iter: int = 1000,
                  col_scale: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None,
                  out: Optional[tuple] = None) -> SolveResult:
    """gpspca_solve_noalloc: the solve with the library's own device scratch (no
    workspace).  `out` = (X (m, p), Z (m, n), support (m, ceil(n/32)) int32)
    preallocated output tensors, else they are allocated here."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    dev = A.device
    nw = (n + 31) // 32
    if out is None:
        out = (torch.empty((m, p), dtype=torch.float32, device=dev),
               torch.empty((m, n), dtype=torch.float32, device=dev),
               torch.empty((m, nw), dtype=torch.int32, device=dev))
    Xt, Zt, sup = out
    if Xt.shape != (m, p) or Zt.shape != (m, n) or sup.shape != (m, nw):
        raise ValueError("output tensors have the wrong shapes")
    trace = (ctypes.c_double * max_iter)()
    nit = ctypes.c_int(0)
    x0p = None
    if X0 is not None:
        X0c = X0.t().contiguous() if X0.dim() == 2 else X0.reshape(1, -1).contiguous()
        if X0c.shape != (m, p) or X0c.dtype != torch.float32:
            raise ValueError("X0 must be a float32 (p, m) tensor")
        x0p = X0c.data_ptr()
    rc = lib.gpspca_solve_noalloc(ctypes.byref(M), form, m, float(gamma), _mu_array(mu, m), x0p,
                                  float(tol), int(max_iter), _stream_ptr(stream), Xt.data_ptr(),
                                  Zt.data_ptr(), sup.data_ptr(), trace, ctypes.byref(nit))
    L.check(rc, "gpspca_solve_noalloc")
    k = nit.value
    return SolveResult(X=Xt.t(), Z=Zt.t(), support=sup, trace=list(trace[:k]), n_iter=k,
                       status=rc)


@dataclass
class StepResult:
    S: torch.Tensor   # (n, m) thresholded correlations
    G: torch.Tensor   # (p, m) float64 ascent direction A S Diag(mu)
    f: list           # per-component objective terms
    nnz: list         # per-component support sizes

    @property
    def F(self) -> float:
        return float(sum(self.f))


def step(A: torch.Tensor, form: int, X: torch.Tensor, gamma: float,
         mu: Optional[Sequence[float]] = None, col_scale: Optional[torch.Tensor] = None,
         stream: Optional[torch.cuda.Stream] = None) -> StepResult:
    """One pass at the feasible point X (p, m) (gpspca_step)."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    Xc = X.reshape(p, -1)
    m = Xc.shape[1]
    Xt = Xc.t().contiguous().to(torch.float32)
    nb = workspace_bytes(A, form, m, 1, col_scale)
    ws = _workspace(nb, A.device)
    St = torch.empty((m, n), dtype=torch.float32, device=A.device)
    Gt = torch.empty((m, p), dtype=torch.float64, device=A.device)
    f = (ctypes.c_double * m)()
    nnz = (ctypes.c_int64 * m)()
    rc = lib.gpspca_step(ctypes.byref(M), form, m, float(gamma), _mu_array(mu, m), Xt.data_ptr(),
                         ws.data_ptr(), ws.numel(), _stream_ptr(stream), St.data_ptr(),
                         Gt.data_ptr(), f, nnz)
    L.check(rc, "gpspca_step")
    return StepResult(S=St.t(), G=Gt.t(), f=list(f), nnz=list(nnz))


def column_norms(A: torch.Tensor, stream: Optional[torch.cuda.Stream] = None,
                 col_scale: Optional[torch.Tensor] = None) -> torch.Tensor:
    lib = L.load()
    M = matrix(A, col_scale)
    out = torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    L.check(lib.gpspca_column_norms(ctypes.byref(M), out.data_ptr(), _stream_ptr(stream)),
            "gpspca_column_norms")
    return out


def profile_enable(on: bool = True, every: int = 1) -> None:
    """Time the dominant kernel's launches with HIP events: the first of each
    solve and every `every`-th after it (False: off)."""
    L.load().gpspca_profile_enable(max(1, int(every)) if on else 0)


def profile_read():
    """(total_ms, launches, kernel name) of the dominant kernel since the last read."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(128)
    L.load().gpspca_profile_read(ctypes.byref(ms), ctypes.byref(cnt), buf, 128)
    return ms.value, cnt.value, buf.value.decode()


@dataclass
class PathResult:
    X: torch.Tensor          # (p, K) column-major view
    Z: torch.Tensor          # (n, K) column-major view
    support: torch.Tensor    # (K, ceil(n/32)) int32 bit words
    traces: list             # per problem: objective F_0 .. F_{n_iter[k]-1}
    n_iter: list
    status: list
    rc: int

    def support_mask(self) -> torch.Tensor:
        return SolveResult(self.X, self.Z, self.support, [], 0, 0).support_mask()


def solve_path(A: torch.Tensor, form: int, gammas: Sequence[float],
               X0: Optional[torch.Tensor] = None, tol: float = 1e-4, max_iter: int = 1000,
               col_scale: Optional[torch.Tensor] = None,
               stream: Optional[torch.cuda.Stream] = None) -> SolveResult:
    """K single-unit problems sharing every pass over A (gpspca_solve_path)."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    K = len(gammas)
    nb = lib.gpspca_path_workspace_bytes(ctypes.byref(M), K, max_iter)
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    ws = _workspace(int(nb), A.device)
    Xt = torch.empty((K, p), dtype=torch.float32, device=A.device)
    Zt = torch.empty((K, n), dtype=torch.float32, device=A.device)
    sup = torch.empty((K, (n + 31) // 32), dtype=torch.int32, device=A.device)
    g = (ctypes.c_double * K)(*[float(v) for v in gammas])
    tr = (ctypes.c_double * (K * max_iter))()
    nit = (ctypes.c_int * K)()
    sts = (ctypes.c_int * K)()
    x0p = None
    if X0 is not None:
        X0c = X0.t().contiguous()
        if X0c.shape != (K, p) or X0c.dtype != torch.float32:
            raise ValueError("X0 must be a float32 (p, K) tensor")
        x0p = X0c.data_ptr()
    rc = lib.gpspca_solve_path(ctypes.byref(M), form, K, g, x0p, float(tol), int(max_iter),
                               ws.data_ptr(), ws.numel(), _stream_ptr(stream), Xt.data_ptr(),
                               Zt.data_ptr(), sup.data_ptr(), tr, nit, sts)
    L.check(rc, "gpspca_solve_path")
    traces = [list(tr[k * max_iter:k * max_iter + nit[k]]) for k in range(K)]
    return PathResult(X=Xt.t(), Z=Zt.t(), support=sup, traces=traces, n_iter=list(nit),
                      status=list(sts), rc=rc)


def solve_multistart(A: torch.Tensor, form: int, m: int, gamma: float, tol: float = 1e-4,
                     max_iter: int = 1000, col_scale: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> PathResult:
    """m single-unit solves with one gamma from the m columns of largest norm,
    sharing every pass over A (gpspca_solve_multistart)."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    nb = lib.gpspca_path_workspace_bytes(ctypes.byref(M), m, max_iter)
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    ws = _workspace(int(nb), A.device)
    Xt = torch.empty((m, p), dtype=torch.float32, device=A.device)
    Zt = torch.empty((m, n), dtype=torch.float32, device=A.device)
    sup = torch.empty((m, (n + 31) // 32), dtype=torch.int32, device=A.device)
    tr = (ctypes.c_double * (m * max_iter))()
    nit = (ctypes.c_int * m)()
    sts = (ctypes.c_int * m)()
    rc = lib.gpspca_solve_multistart(ctypes.byref(M), form, m, float(gamma), float(tol),
                                     int(max_iter), ws.data_ptr(), ws.numel(),
                                     _stream_ptr(stream), Xt.data_ptr(), Zt.data_ptr(),
                                     sup.data_ptr(), tr, nit, sts)
    L.check(rc, "gpspca_solve_multistart")
    traces = [list(tr[k * max_iter:k * max_iter + nit[k]]) for k in range(m)]
    return PathResult(X=Xt.t(), Z=Zt.t(), support=sup, traces=traces, n_iter=list(nit),
                      status=list(sts), rc=rc)


def solve_deflated(A: torch.Tensor, form: int, m: int, gamma: float, tol: float = 1e-4,
                   max_iter: int = 1000,
                   stream: Optional[torch.cuda.Stream] = None) -> PathResult:
    """m single-unit components by projection deflation, component k solved on
    (I - X_{<k} X_{<k}^T) A from that matrix's default start
    (gpspca_solve_deflated; FP32 A)."""
    lib = L.load()
    M = matrix(A)
    p, n = A.shape
    nb = lib.gpspca_deflated_workspace_bytes(ctypes.byref(M), m, max_iter)
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    ws = _workspace(int(nb), A.device)
    Xt = torch.empty((m, p), dtype=torch.float32, device=A.device)
    Zt = torch.empty((m, n), dtype=torch.float32, device=A.device)
    sup = torch.empty((m, (n + 31) // 32), dtype=torch.int32, device=A.device)
    tr = (ctypes.c_double * (m * max_iter))()
    nit = (ctypes.c_int * m)()
    sts = (ctypes.c_int * m)()
    rc = lib.gpspca_solve_deflated(ctypes.byref(M), form, m, float(gamma), float(tol),
                                   int(max_iter), ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                                   Xt.data_ptr(), Zt.data_ptr(), sup.data_ptr(), tr, nit, sts)
    L.check(rc, "gpspca_solve_deflated")
    traces = [list(tr[k * max_iter:k * max_iter + nit[k]]) for k in range(m)]
    return PathResult(X=Xt.t(), Z=Zt.t(), support=sup, traces=traces, n_iter=list(nit),
                      status=list(sts), rc=rc)


def quantize(A: torch.Tensor, dtype: torch.dtype, stream: Optional[torch.cuda.Stream] = None):
    """Reduced-precision copy of the FP32 device matrix A (p, n) (gpspca_quantize).

    dtype torch.bfloat16 (round to nearest even, scale 1) or torch.float8_e4m3fn
    (per-column scale max|a|/448, round to nearest even, saturating).  Returns
    (Aq, scale): Aq is a (p, n) column-major view with a leading dimension padded
    to a multiple of 16 elements; scale is an (n,) FP32 tensor (None for bfloat16)."""
    lib = L.load()
    if dtype not in (torch.bfloat16, torch.float8_e4m3fn):
        raise ValueError("dtype must be torch.bfloat16 or torch.float8_e4m3fn")
    M = matrix(A)
    p, n = A.shape
    ldq = (p + 15) // 16 * 16
    store = torch.zeros((n, ldq), dtype=dtype, device=A.device)
    scale = torch.empty(n, dtype=torch.float32, device=A.device) \
        if dtype == torch.float8_e4m3fn else None
    to = L.BF16 if dtype == torch.bfloat16 else L.F8E4M3
    L.check(lib.gpspca_quantize(ctypes.byref(M), to, store.data_ptr(), ldq,
                                None if scale is None else scale.data_ptr(), _stream_ptr(stream)),
            "gpspca_quantize")
    return store[:, :p].t(), scale


def refine(A: torch.Tensor, form: int, m: int, gamma: float, support: torch.Tensor,
           X0: torch.Tensor, mu: Optional[Sequence[float]] = None, tol: float = 0.0,
           max_iter: int = 5, stream: Optional[torch.cuda.Stream] = None) -> SolveResult:
    """FP32 passes restricted to a frozen support (gpspca_refine): `support` is the
    (m, ceil(n/32)) int32 word tensor of a previous result, X0 its (p, m) iterate."""
    lib = L.load()
    M = matrix(A)
    p, n = A.shape
    dev = A.device
    nb = workspace_bytes(A, form, m, max_iter)
    ws = _workspace(nb, dev)
    Xt = torch.empty((m, p), dtype=torch.float32, device=dev)
    Zt = torch.empty((m, n), dtype=torch.float32, device=dev)
    sup = torch.empty((m, (n + 31) // 32), dtype=torch.int32, device=dev)
    sin = support.contiguous()
    X0c = X0.reshape(p, -1).t().contiguous().to(torch.float32)
    if sin.shape != (m, (n + 31) // 32) or X0c.shape != (m, p):
        raise ValueError("support must be (m, ceil(n/32)) words and X0 (p, m)")
    trace = (ctypes.c_double * max_iter)()
    nit = ctypes.c_int(0)
    rc = lib.gpspca_refine(ctypes.byref(M), form, m, float(gamma), _mu_array(mu, m),
                           sin.data_ptr(), X0c.data_ptr(), float(tol), int(max_iter),
                           ws.data_ptr(), ws.numel(), _stream_ptr(stream), Xt.data_ptr(),
                           Zt.data_ptr(), sup.data_ptr(), trace, ctypes.byref(nit))
    L.check(rc, "gpspca_refine")
    k = nit.value
    return SolveResult(X=Xt.t(), Z=Zt.t(), support=sup, trace=list(trace[:k]), n_iter=k,
                       status=rc)


def refine_path(A: torch.Tensor, form: int, gammas: Sequence[float], support: torch.Tensor,
                X0: torch.Tensor, tol: float = 0.0, max_iter: int = 5,
                stream: Optional[torch.cuda.Stream] = None) -> PathResult:
    """gpspca_refine_path: each of the K problems restricted to its own support."""
    lib = L.load()
    M = matrix(A)
    p, n = A.shape
    K = len(gammas)
    nb = lib.gpspca_path_workspace_bytes(ctypes.byref(M), K, max_iter)
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    ws = _workspace(int(nb), A.device)
    Xt = torch.empty((K, p), dtype=torch.float32, device=A.device)
    Zt = torch.empty((K, n), dtype=torch.float32, device=A.device)
    sup = torch.empty((K, (n + 31) // 32), dtype=torch.int32, device=A.device)
    sin = support.contiguous()
    X0c = X0.t().contiguous().to(torch.float32)
    if sin.shape != (K, (n + 31) // 32) or X0c.shape != (K, p):
        raise ValueError("support must be (K, ceil(n/32)) words and X0 (p, K)")
    g = (ctypes.c_double * K)(*[float(v) for v in gammas])
    tr = (ctypes.c_double * (K * max_iter))()
    nit = (ctypes.c_int * K)()
    sts = (ctypes.c_int * K)()
    rc = lib.gpspca_refine_path(ctypes.byref(M), form, K, g, sin.data_ptr(), X0c.data_ptr(),
                                float(tol), int(max_iter), ws.data_ptr(), ws.numel(),
                                _stream_ptr(stream), Xt.data_ptr(), Zt.data_ptr(),
                                sup.data_ptr(), tr, nit, sts)
    L.check(rc, "gpspca_refine_path")
    traces = [list(tr[k * max_iter:k * max_iter + nit[k]]) for k in range(K)]
    return PathResult(X=Xt.t(), Z=Zt.t(), support=sup, traces=traces, n_iter=list(nit),
                      status=list(sts), rc=rc)


def autotune(A: torch.Tensor, form: int, m: int, gamma: float, X0: Optional[torch.Tensor] = None,
             passes: int = 3, col_scale: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> dict:
    """Time the correlation-kernel configurations for this problem and record the
    fastest for later solves (gpspca_autotune).  X0 (p, m) defaults to the first m
    columns of the identity; form SL1/SL0 with m > 1 tunes a gamma path."""
    lib = L.load()
    M = matrix(A, col_scale)
    p, n = A.shape
    if X0 is None:
        X0 = torch.zeros((p, m), dtype=torch.float32, device=A.device)
        X0[torch.arange(m), torch.arange(m)] = 1.0
    X0c = X0.reshape(p, -1).t().contiguous().to(torch.float32)
    path = form in (L.SL1, L.SL0) and m > 1
    nb = (lib.gpspca_path_workspace_bytes(ctypes.byref(M), m, passes + 1) if path
          else lib.gpspca_workspace_bytes(ctypes.byref(M), form, m, passes + 1))
    if nb == 0:
        raise L.GpspcaError(L.EINVAL, L.last_error())
    ws = _workspace(int(nb), A.device)
    nt = ctypes.c_int(0)
    best = ctypes.c_double(0.0)
    desc = ctypes.create_string_buffer(128)
    L.check(lib.gpspca_autotune(ctypes.byref(M), form, m, float(gamma), X0c.data_ptr(), passes,
                                ws.data_ptr(), ws.numel(), _stream_ptr(stream), ctypes.byref(nt),
                                ctypes.byref(best), desc, 128), "gpspca_autotune")
    return {"timed": nt.value, "best_ms_per_pass": best.value, "choice": desc.value.decode()}


def autotune_clear() -> None:
    L.load().gpspca_autotune_clear()
