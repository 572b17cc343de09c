"""Helpers shared by the GPU parity tests: device transfer, the FP32 tie band of
the correlation, and gamma selection away from ties.  Expected values always
come from the oracle (never from the GPU path)."""
from __future__ import annotations

import math

import numpy as np

import oracle as O

FORM_NAMES = {O.SL1: "SL1", O.SL0: "SL0", O.BL1: "BL1", O.BL0: "BL0"}


def is_l0(form: int) -> bool:
    return form in (O.SL0, O.BL0)


def to_device(A: np.ndarray, lda: int | None = None, dtype=None):
    """Column-major device copy of A (p, n) as a torch (p, n) view with stride (1, lda)."""
    import torch
    p, n = A.shape
    lda = p if lda is None else lda
    buf = np.zeros((n, lda), dtype=np.float32 if dtype is None else dtype)
    buf[:, :p] = A.T
    t = torch.from_numpy(buf).cuda()
    return t[:, :p].t()


def x_to_device(X: np.ndarray):
    import torch
    X = np.asarray(X, dtype=np.float32).reshape(X.shape[0], -1)
    return torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t()


def chain_depth(p: int) -> float:
    """lambda sqrt(L) with lambda = 4 and L = ceil(p/4) + 64, an upper bound on
    the longest chain of FP32 additions in one correlation on the GPU (the
    matrix-core kernels carry one accumulator through p/4 steps of four
    products; the other kernels use shorter per-lane chains and a tree).

    This is a probabilistic bound, not a worst-case one: for rounding errors
    modelled as independent and mean-zero, a sum along a chain of L additions
    errs by at most lambda sqrt(L) u sum|terms| (u = 2^-24) except with
    probability about 2 exp(-lambda^2 / 2) (Higham and Mary, SIAM J. Sci.
    Comput. 41(5), 2019).  The deterministic bound L u sum|terms| is sqrt(L)/4
    times wider (about 12x at p = 10^4) and would mark far more elements as
    ties.  Every use multiplies the band by a safety factor of 4 or 8, so the
    effective lambda is 16 or more."""
    return 4.0 * math.sqrt(math.ceil(p / 4) + 64)


def corr_band(A64: np.ndarray, X64: np.ndarray) -> np.ndarray:
    """Probabilistic error bound of the FP32 correlation a_i^T x_j (n x m):
    chain_depth(p) u sum_r |A_ri X_rj|."""
    p = A64.shape[0]
    return chain_depth(p) * 2.0 ** -24 * (np.abs(A64).T @ np.abs(X64)) + 1e-30


def margins(Y: np.ndarray, form: int, gamma: float, mu: np.ndarray):
    """Threshold margin per element and its band given the correlation band."""
    if is_l0(form):
        return (mu[None, :] * Y) ** 2 - gamma
    return mu[None, :] * np.abs(Y) - gamma


def margin_band(Y: np.ndarray, eb: np.ndarray, form: int, mu: np.ndarray):
    if is_l0(form):
        return mu[None, :] ** 2 * (2 * np.abs(Y) * eb + eb * eb)
    return mu[None, :] * eb


def term_band(A64, X64, S64, form, mu):
    """FP32 band of each component's objective term f_j (length m): f_j sums
    t^2 (l1, t = mu|y| - gamma) or q = (mu y)^2 - gamma (l0) over the support,
    and each summand moves by its margin's band when y does (2 t mu e + (mu e)^2
    for l1, the margin band itself for l0).  A small f_j that is a difference of
    large numbers keeps only this absolute accuracy."""
    m = X64.shape[1]
    mu = np.ones(m) if mu is None else np.asarray(mu, dtype=np.float64)
    Y = A64.T @ X64
    eb = corr_band(A64, X64)
    on = S64 != 0
    if is_l0(form):
        per = margin_band(Y, eb, form, mu)
    else:
        t = np.abs(S64)
        per = 2.0 * t * mu[None, :] * eb + (mu[None, :] * eb) ** 2
    return (per * on).sum(axis=0)


def trajectory(A64, form, m, gamma, mu, X0, iters):
    """Oracle iterates X_0..X_{iters-1} (composition of oracle.step / oracle.retract)."""
    Xs = [np.asfortranarray(X0)]
    X = Xs[0]
    for _ in range(iters - 1):
        st = O.step(A64, form, X, gamma, mu=None if m == 1 and form < 2 else mu)
        if st["F"] == 0.0:
            break
        X, _ = O.retract(st["G"], st["nnz"], X)
        Xs.append(X)
    return Xs


def pick_gamma(A64, form, m, mu, X0, gamma0, iters=1, safety=8.0, tries=60):
    """l0 forms: smallest nudge of gamma0 (multiplicative, deterministic) such that
    at every oracle iterate no threshold margin lies within `safety` x its FP32
    band -- a hard threshold that flips moves G by mu*y*a_i, so l0 parity needs
    no ties.  l1 forms: gamma0 unchanged -- the soft threshold is continuous
    (s is within the band of 0 on both sides of a tie), so ties are excluded
    from the support comparison instead (tie_mask)."""
    if not is_l0(form):
        return gamma0
    mu = np.ones(m) if mu is None else np.asarray(mu, dtype=np.float64)
    for k in range(tries):
        g = gamma0 * (1.0 + 0.0137 * k) if k else gamma0
        ok = True
        for X in trajectory(A64, form, m, g, mu, X0, iters):
            Y = A64.T @ X
            eb = corr_band(A64, X)
            if np.any(np.abs(margins(Y, form, g, mu)) <= safety * margin_band(Y, eb, form, mu)):
                ok = False
                break
        if ok:
            return g
    raise RuntimeError("could not place gamma away from ties")


def pick_gamma_starts(A64, form, x0s, gamma0, iters=1):
    """pick_gamma for several single-unit starts at once (multi-start solves):
    a gamma whose trajectories from every start stay away from ties."""
    g = gamma0
    for _ in range(8):
        g_prev = g
        for x0 in x0s:
            g = pick_gamma(A64, form, 1, None, x0, g, iters=iters)
        if g == g_prev:
            return g
    raise RuntimeError("could not place gamma away from ties for every start")


def fp32_round(X: np.ndarray) -> np.ndarray:
    return np.asarray(X, dtype=np.float32).astype(np.float64)


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def tie_mask(A64, X64, form, gamma, mu, safety=4.0):
    """Elements (n x m) whose threshold margin at X lies within `safety` x the FP32
    band: there the GPU and the oracle may legitimately decide differently."""
    m = X64.shape[1]
    mu = np.ones(m) if mu is None else np.asarray(mu, dtype=np.float64)
    Y = A64.T @ X64
    eb = corr_band(A64, X64)
    return np.abs(margins(Y, form, gamma, mu)) <= safety * margin_band(Y, eb, form, mu)


TNAME = {O.BF16: "bf16", O.E4M3: "e4m3"}


def _torch_dtype(to):
    import torch
    return {O.BF16: torch.bfloat16, O.E4M3: torch.float8_e4m3fn}[to]


class _TorchDtypes(dict):
    """O.BF16 / O.E4M3 -> torch dtype, resolved on first use (torch is imported lazily)."""

    def __missing__(self, to):
        v = _torch_dtype(to)
        self[to] = v
        return v


TD = _TorchDtypes()


def q_to_device(codes, to, p):
    """Device (p, n) view of oracle codes (ldq x n, column-major)."""
    import torch
    ldq, n = codes.shape
    host = np.ascontiguousarray(codes.T)
    t = torch.from_numpy(host.view(np.int16) if to == O.BF16 else host).cuda()
    t = t.view(TD[to])
    return t[:, :p].t()


def quantized_problem(p, n, m, seed, to, ldq_pad=0, A32=None):
    """A planted FP32 matrix (or the given one), the oracle's codes of it on the
    device, their dequantized FP64 values and the device column scales."""
    import torch
    from workloads import generators as W
    if A32 is None:
        A32, _, _ = W.planted_block(p, n, max(1, min(m, 4)), seed, k=min(40, n // 8))
    align = 8 if to == O.BF16 else 16
    ldq = (p + align - 1) // align * align + ldq_pad * align
    codes, scale = O.quantize(A32, to, ldq=ldq)
    Adeq = O.dequantize(codes, to, scale, p)
    Ad = q_to_device(codes, to, p)
    sc = torch.from_numpy(scale).cuda() if to == O.E4M3 else None
    return A32, Adeq, Ad, sc
