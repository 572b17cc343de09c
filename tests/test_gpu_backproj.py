"""Back-projection G = A S N (Section 2, Table 1) on the matrix cores (the
dense form of k_backproj and k_backproj_dense) against the FP64 oracle.

A pass is back-projected densely on the matrix cores when enough of its
columns are active, else over the active columns only
(k_backproj); one decision covers the whole pass.  Each test forces one of
the two (GPSPCA_BACKPROJ=dense|sparse) or a threshold at which both kernels
take ranges of one pass.

Shapes cover:
- ragged row quads (p % 4 = 1, 2, 3) and several row blocks;
- column ranges whose length is not a multiple of the 4-column step;
- 1, 2 and 4 component groups of 16;
- FP32, BF16 and e4m3 storage;
- block solves and gamma paths.

G and the objective match to 1e-5 relative, like every other pass kernel; S
and the supports are the correlation kernel's and must match exactly away
from ties."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, TNAME, fp32_round, is_l0, pick_gamma, quantized_problem, rel,
                   tie_mask, to_device, x_to_device)

pytestmark = pytest.mark.gpu

# (form, m, p, n, lda, seed); lda % 4 == 0 (the matrix-core kernel's loads)
CASES = [
    (O.BL1, 5, 1003, 3001, 1004, 1),     # p % 4 = 3, one component group
    (O.BL1, 16, 2048, 2999, 2048, 2),
    (O.BL1, 17, 257, 4001, 260, 3),      # p % 4 = 1, two groups (one partial)
    (O.BL1, 32, 12002, 1203, 12004, 4),  # p % 4 = 2, 47 row blocks
    (O.BL1, 40, 515, 2000, 516, 5),      # three groups (four-group kernel)
    (O.BL1, 64, 700, 1501, 700, 6),
    (O.BL0, 18, 400, 800, 400, 7),
]


def _ids(c):
    return f"{FORM_NAMES[c[0]]}-m{c[1]}-p{c[2]}-n{c[3]}-lda{c[4]}"


def _problem(case):
    form, m, p, n, lda, seed = case
    A32, _, _ = W.planted_block(p, n, min(m, 4), seed, k=min(50, n // 8))
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.6, m)
    X0 = fp32_round(O.init(A64, m)[0])
    # small gammas: most columns active, so the dense kernel takes every range
    g0 = W.gamma_absolute(A64, is_l0(form), 0.002 if is_l0(form) else 0.01)
    gamma = pick_gamma(A64, form, m, mu, X0, g0, iters=1)
    return A32, A64, mu, X0, gamma


def _check_step(out, ref, A64, X0, form, gamma, mu):
    S = out.S.cpu().numpy().astype(np.float64)
    ties = tie_mask(A64, X0, form, gamma, mu)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_dense_step_parity(gpu, case, monkeypatch):
    form, m, p, n, lda, seed = case
    print(f"\n[backproj dense] {_ids(case)}", flush=True)
    A32, A64, mu, X0, gamma = _problem(case)
    Ad = to_device(A32, lda=lda)
    ref = O.step(A64, form, X0, gamma, mu=mu)
    assert (ref["S"] != 0).any(axis=1).mean() > 0.5
    monkeypatch.setenv("GPSPCA_BACKPROJ", "dense")
    dense = gpu.step(Ad, form, x_to_device(X0), gamma, mu=list(mu))
    _check_step(dense, ref, A64, X0, form, gamma, mu)
    monkeypatch.setenv("GPSPCA_BACKPROJ", "sparse")
    sparse = gpu.step(Ad, form, x_to_device(X0), gamma, mu=list(mu))
    _check_step(sparse, ref, A64, X0, form, gamma, mu)
    np.testing.assert_array_equal(dense.S.cpu().numpy(), sparse.S.cpu().numpy())


@pytest.mark.parametrize("m", [8, 32])
def test_mixed_dense_and_sparse_ranges(gpu, m, monkeypatch):
    """Strong columns in the first 40% of A and weak ones after.  When the pass
    is dense (threshold 300/1024 of the columns active), the ranges with
    active columns, the one that straddles the boundary included, go to the
    matrix-core kernel and the empty ones to the support-restricted kernel."""
    p, n = 1001, 20000
    rng = np.random.default_rng(50 + m)
    A32 = (rng.standard_normal((p, n)) * 0.01).astype(np.float32)
    A32[:, : 2 * n // 5] *= 100.0
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.8, m)
    X0 = fp32_round(O.init(A64, m)[0])
    gamma = 0.5 * float(np.median(np.abs(A64[:, : 2 * n // 5].T @ X0)))
    ref = O.step(A64, O.BL1, X0, gamma, mu=mu)
    act = (ref["S"] != 0).any(axis=1)
    assert act[: 2 * n // 5].mean() > 0.8 and act[2 * n // 5:].mean() < 0.01
    Ad = to_device(A32, lda=1004)
    for mode in ("auto", "300"):
        monkeypatch.setenv("GPSPCA_BACKPROJ", mode)
        out = gpu.step(Ad, O.BL1, x_to_device(X0), gamma, mu=list(mu))
        _check_step(out, ref, A64, X0, O.BL1, gamma, mu)


@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
@pytest.mark.parametrize("m,p,n", [(12, 1001, 3001), (33, 2050, 1999)])
def test_dense_step_quantized(gpu, to, m, p, n, monkeypatch):
    print(f"\n[backproj dense] {TNAME[to]} m={m} p={p} n={n}", flush=True)
    A32, Adeq, Ad, sc = quantized_problem(p, n, m, 60 + m, to)
    mu = np.linspace(1.0, 0.7, m)
    X0 = fp32_round(O.init(Adeq, m)[0])
    gamma = W.gamma_absolute(Adeq, False, 0.01)
    ref = O.step(Adeq, O.BL1, X0, gamma, mu=mu)
    monkeypatch.setenv("GPSPCA_BACKPROJ", "dense")
    out = gpu.step(Ad, O.BL1, x_to_device(X0), gamma, mu=list(mu), col_scale=sc)
    _check_step(out, ref, Adeq, X0, O.BL1, gamma, mu)


@pytest.mark.parametrize("mode", ["dense", "auto"])
def test_dense_block_solve(gpu, mode, monkeypatch):
    form, m, p, n, lda, seed = (O.BL1, 20, 1503, 5001, 1504, 9)
    A32, A64, mu, X0, gamma = _problem((form, m, p, n, lda, seed))
    monkeypatch.setenv("GPSPCA_BACKPROJ", mode)
    rs = O.solve(A64, form, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=8)
    res = gpu.solve(to_device(A32, lda=lda), form, m, gamma, mu=list(mu), X0=x_to_device(X0),
                    tol=0.0, max_iter=8)
    assert res.n_iter == rs["n_iter"]
    np.testing.assert_allclose(res.trace, rs["trace"], rtol=1e-5)
    assert rel(res.X.cpu().numpy(), rs["X"]) <= 1e-5


@pytest.mark.parametrize("form", [O.SL1, O.SL0])
@pytest.mark.parametrize("K", [16, 32, 64])
def test_dense_gamma_path(gpu, form, K, monkeypatch):
    """K single-unit problems at log-spaced gammas: at the small ones nearly
    every column is active, so the dense kernel takes the back-projection of
    the whole batch."""
    p, n, iters = 1002, 6001, 6
    print(f"\n[backproj path] {FORM_NAMES[form]} K={K}", flush=True)
    A32, _, _, _ = W.planted_single(p, n, 70 + K, k=40)
    A64 = A32.astype(np.float64)
    x0 = fp32_round(O.init(A64, 1)[0])
    fr = W.gamma_fractions(K, 0.01, 0.5) if not is_l0(form) else W.gamma_fractions(K, 0.003, 0.05)
    gammas = [W.gamma_absolute(A64, is_l0(form), f) for f in fr]
    check = sorted({0, K // 3, K - 1})
    for k in check:
        gammas[k] = pick_gamma(A64, form, 1, None, x0, gammas[k], iters=iters)
    monkeypatch.setenv("GPSPCA_BACKPROJ", "dense")
    res = gpu.solve_path(to_device(A32, lda=1004), form, gammas,
                         X0=x_to_device(np.repeat(x0, K, axis=1)), tol=0.0, max_iter=iters)
    X = res.X.cpu().numpy()
    for k in check:
        ref = O.solve(A64, form, 1, gammas[k], X0=x0, tol=0.0, max_iter=iters)
        assert res.n_iter[k] == ref["n_iter"]
        np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
        if ref["trace"][-1] != 0.0:
            assert rel(X[:, k], ref["X"][:, 0]) <= 1e-5
