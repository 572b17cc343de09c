"""Seeded synthetic inputs for the GP-SPCA power iteration.

This module only draws random matrices and the planted structure of the test
workloads.  It holds none of the arithmetic of the method itself (no
correlation, threshold, back-projection or retraction), so that both the FP64
oracle and the GPU path can be fed identical inputs without sharing code.

Storage convention: a data matrix A in R^{p x n} (p samples, n variables,
Section 2 of the paper) is returned as a NumPy array of shape (p, n) in
Fortran (column-major) order, so that every variable column a_i is contiguous.

Every draw is made per chunk of ``CHUNK`` columns from its own child seed of
``numpy.random.SeedSequence(seed)``, so the values do not depend on how many
threads generate them.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 4096


def _threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return min(int(env), 16)
    return min(os.cpu_count() or 1, 16)


def _noise(p: int, n: int, seed: int, dtype) -> np.ndarray:
    """i.i.d. N(0,1) entries, drawn column-chunk by column-chunk."""
    A = np.empty((p, n), dtype=dtype, order="F")
    nchunk = (n + CHUNK - 1) // CHUNK
    kids = np.random.SeedSequence(seed).spawn(nchunk + 1)

    def fill(c: int) -> None:
        c0, c1 = c * CHUNK, min(n, (c + 1) * CHUNK)
        rng = np.random.default_rng(kids[c])
        # Column-major block: draw as (cols, p) rows then view transposed.
        blk = rng.standard_normal((c1 - c0, p), dtype=np.float64 if dtype == np.float64 else np.float32)
        A[:, c0:c1] = blk.T

    if nchunk == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nchunk)))
    return A


def _structure_rng(seed: int) -> np.random.Generator:
    """Generator for the planted structure, independent of the noise chunks."""
    return np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))


def gaussian_centered(p: int, n: int, seed: int) -> np.ndarray:
    """FP64 N(0,1) matrix with every column centred over its p rows.

    Small oracle-scale workload (p=100, n=1000 in the reference setting)."""
    A = _noise(p, n, seed, np.float64)
    A -= A.mean(axis=0, keepdims=True)
    return np.asfortranarray(A)


def gaussian(p: int, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Plain i.i.d. N(0,1) matrix (no planted structure)."""
    return _noise(p, n, seed, dtype)


def planted_single(p: int, n: int, seed: int, k: int = 500, beta: float | None = None,
                   dtype=np.float32):
    """Single-spike model: A = noise + sqrt(beta) * u v^T.

    u is a unit Gaussian direction in R^p; v is a k-sparse unit vector with
    entries +-1/sqrt(k) on k indices drawn without replacement; beta defaults
    to 5*sqrt(n).  Returns (A, u, v_support, v_values)."""
    if beta is None:
        beta = 5.0 * math.sqrt(n)
    k = min(k, n)
    A = _noise(p, n, seed, dtype)
    rng = _structure_rng(seed)
    g = rng.standard_normal(p)
    u = g / np.linalg.norm(g)
    idx = np.sort(rng.choice(n, size=k, replace=False))
    vals = rng.choice(np.array([-1.0, 1.0]), size=k) / math.sqrt(k)
    sb = math.sqrt(beta)
    for i, v in zip(idx, vals):
        A[:, i] = (A[:, i].astype(np.float64) + sb * v * u).astype(dtype)
    return A, u, idx, vals


def planted_block(p: int, n: int, m: int, seed: int, k: int = 200, dtype=np.float32):
    """m planted components: A = noise + sum_j sqrt(beta_j) u_j v_j^T.

    U = [u_1..u_m] is the Q factor of a p x m Gaussian matrix (diag(R) > 0);
    the v_j are k-sparse with disjoint supports taken from one random
    permutation, entries +-1/sqrt(k); beta_j = 5*sqrt(n)/j.
    Returns (A, U, supports) where supports[j] holds v_j's indices."""
    A = _noise(p, n, seed, dtype)
    rng = _structure_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((p, m)))
    Q = Q * np.sign(np.diag(R))[None, :]
    k = min(k, n // max(m, 1))
    perm = rng.permutation(n)
    supports = []
    for j in range(m):
        idx = np.sort(perm[j * k:(j + 1) * k])
        vals = rng.choice(np.array([-1.0, 1.0]), size=k) / math.sqrt(k)
        sb = math.sqrt(5.0 * math.sqrt(n) / (j + 1))
        for i, v in zip(idx, vals):
            A[:, i] = (A[:, i].astype(np.float64) + sb * v * Q[:, j]).astype(dtype)
        supports.append(idx)
    return A, Q, supports


def gamma_fractions(count: int, lo: float = 0.01, hi: float = 0.5) -> np.ndarray:
    """Log-spaced sparsity fractions from lo to hi (both included)."""
    if count == 1:
        return np.array([lo])
    return np.exp(np.linspace(math.log(lo), math.log(hi), count))


def gamma_absolute(A: np.ndarray, l0: bool, frac: float) -> float:
    """Workload convention: gamma as a fraction of the largest column norm
    (L1 penalties) or of its square (L0 penalties)."""
    cmax = float(np.sqrt((A.astype(np.float64) ** 2).sum(axis=0)).max())
    return frac * (cmax * cmax if l0 else cmax)


def random_orthonormal(p: int, m: int, seed: int) -> np.ndarray:
    """A p x m matrix with orthonormal columns (Q factor of a Gaussian draw)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x0B]))
    Q, R = np.linalg.qr(rng.standard_normal((p, m)))
    return np.asfortranarray(Q * np.sign(np.diag(R))[None, :])


def serving_requests(count: int, seed: int = 1000, p_max: int = 20000, n_max: int = 200000,
                     repeat: float = 0.5):
    """Request descriptors of the mixed serving workload.

    p log-uniform in [200, p_max], n log-uniform in [2000, n_max] (20000 and
    200000 in the full setting), a formulation uniform over the four, m in
    {1, 4, 16} (for a single-unit form, m > 1 means m starts from the m columns
    of largest norm), gamma fraction uniform in
    [0.01, 0.5], storage FP32 or bfloat16 (even odds), and with probability
    `repeat` a repeat of an earlier request's matrix (a new gamma, form and m
    on a matrix that may still be resident)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        if out and rng.random() < repeat:
            prev = out[int(rng.integers(len(out)))]
            p, n, mseed, dt = prev["p"], prev["n"], prev["matrix_seed"], prev["dtype"]
        else:
            p = int(round(math.exp(rng.uniform(math.log(200), math.log(p_max)))))
            n = int(round(math.exp(rng.uniform(math.log(2000), math.log(n_max)))))
            mseed = seed + r
            dt = "f32" if rng.random() < 0.5 else "bf16"
        form = int(rng.integers(4))
        m = int(rng.choice([1, 4, 16]))
        m = min(m, p)
        frac = float(rng.uniform(0.01, 0.5))
        out.append(dict(p=p, n=n, matrix_seed=mseed, dtype=dt, form=form, m=m, frac=frac))
    return out
