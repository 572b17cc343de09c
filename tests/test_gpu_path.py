"""Gamma path (gpspca_solve_path): K single-unit problems sharing each pass over
A.  Column k must equal the FP64 oracle's single-unit solve with gamma_k from
the same start (same stopping pass, X, Z, trace within 1e-5, supports equal
outside the FP32 tie band), and the library's own single solve."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (fp32_round, is_l0, pick_gamma, pick_gamma_starts, rel, tie_mask, to_device,
                   x_to_device)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form,K,p,n,lda_extra", [
    (O.SL1, 8, 600, 4000, 0),
    (O.SL0, 8, 600, 4000, 0),
    (O.SL1, 32, 1001, 3000, 3),
    (O.SL0, 5, 257, 2000, 1),
    # more tiles of 16 columns than matrix-core waves: the leftover tiles are
    # split by rows (two component groups)
    (O.SL1, 32, 300, 20000, 0),
])
def test_path_columns_match_single_solves(gpu, form, K, p, n, lda_extra):
    print(f"\n[path] form={form} K={K} p={p} n={n}", flush=True)
    A32, _, _, _ = W.planted_single(p, n, 11, k=60)
    A64 = A32.astype(np.float64)
    x0 = fp32_round(O.init(A64, 1)[0])
    fr = W.gamma_fractions(K, 0.01, 0.5) if not is_l0(form) else W.gamma_fractions(K, 0.003, 0.05)
    iters = 10
    gammas = [pick_gamma(A64, form, 1, None, x0, W.gamma_absolute(A64, is_l0(form), f), iters=iters)
              for f in fr]
    # a tolerance that no column's relative objective change comes near, so the
    # per-column stopping decisions are far from their threshold
    ratios = []
    for g in gammas:
        tr = O.solve(A64, form, 1, g, X0=x0, tol=0.0, max_iter=iters)["trace"]
        ratios += list(np.abs(np.diff(tr)) / np.maximum(np.abs(tr[:-1]), 1e-300))
    ratios = np.array(ratios)
    tol = next(t for t in (3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 0.0)
               if t == 0.0 or not np.any((ratios > t / 2) & (ratios < 2 * t)))
    Ad = to_device(A32, lda=p + lda_extra)
    res = gpu.solve_path(Ad, form, gammas, X0=x_to_device(np.repeat(x0, K, axis=1)), tol=tol,
                         max_iter=iters)
    X = res.X.cpu().numpy().astype(np.float64)
    Z = res.Z.cpu().numpy().astype(np.float64)
    sup = res.support_mask().cpu().numpy()
    for k, g in enumerate(gammas):
        ref = O.solve(A64, form, 1, g, X0=x0, tol=tol, max_iter=iters)
        assert res.n_iter[k] == ref["n_iter"], k
        assert res.status[k] == ref["status"], k
        np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
        if ref["trace"][-1] == 0.0:
            assert not sup[:, k].any()
            continue
        assert rel(X[:, k], ref["X"][:, 0]) <= 1e-5
        assert rel(Z[:, k], ref["Z"][:, 0]) <= 1e-5
        ties = tie_mask(A64, ref["X"], form, g, None)[:, 0]
        np.testing.assert_array_equal(sup[~ties, k], ref["support"][~ties, 0])


def test_path_default_start_and_single_solve_agree(gpu):
    p, n, K = 800, 5000, 6
    A32, _, _, _ = W.planted_single(p, n, 12, k=80)
    A64 = A32.astype(np.float64)
    cmax = np.sqrt((A64 ** 2).sum(axis=0)).max()
    gammas = list(cmax * np.array([0.02, 0.04, 0.08, 0.12, 0.2, 1.5]))  # last one: empty support
    Ad = to_device(A32)
    res = gpu.solve_path(Ad, O.SL1, gammas, tol=0.0, max_iter=8)
    for k, g in enumerate(gammas):
        single = gpu.solve(Ad, O.SL1, 1, g, tol=0.0, max_iter=8)
        assert res.n_iter[k] == single.n_iter
        np.testing.assert_allclose(res.traces[k], single.trace, rtol=1e-5)
        assert rel(res.X[:, k].cpu().numpy(), single.X[:, 0].cpu().numpy()) <= 1e-5
    assert res.status[-1] == O.DEGENERATE and res.traces[-1] == [0.0]


@pytest.mark.parametrize("form,m,p,n", [(O.SL1, 5, 601, 3001), (O.SL0, 16, 257, 2000),
                                        (O.SL1, 1, 300, 900)])
def test_multistart_columns_match_single_solves(gpu, form, m, p, n):
    """gpspca_solve_multistart: problem k starts at the column of the k-th
    largest norm (ties to the lower index), normalized, and equals the oracle's
    single-unit solve from there."""
    print(f"\n[multistart] form={form} m={m} p={p} n={n}", flush=True)
    A32, _, _, _ = W.planted_single(p, n, 31 + m, k=50)
    A64 = A32.astype(np.float64)
    idx = O.top_m(O.column_norms(A64), m)
    frac = 0.1 if not is_l0(form) else 0.02
    g = W.gamma_absolute(A64, is_l0(form), frac)
    x0s = [fp32_round(A64[:, [i]] / np.linalg.norm(A64[:, i])) for i in idx]
    iters = 8
    g = pick_gamma_starts(A64, form, x0s, g, iters=iters)
    res = gpu.solve_multistart(to_device(A32), form, m, g, tol=0.0, max_iter=iters)
    X = res.X.cpu().numpy().astype(np.float64)
    sup = res.support_mask().cpu().numpy()
    for k in range(m):
        ref = O.solve(A64, form, 1, g, X0=x0s[k], tol=0.0, max_iter=iters)
        assert res.n_iter[k] == ref["n_iter"] and res.status[k] == ref["status"], k
        np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
        if ref["trace"][-1] == 0.0:
            continue
        assert rel(X[:, k], ref["X"][:, 0]) <= 1e-5
        ties = tie_mask(A64, ref["X"], form, g, None)[:, 0]
        np.testing.assert_array_equal(sup[~ties, k], ref["support"][~ties, 0])


def test_multistart_argument_checks(gpu):
    import paper_1312_6182_amd as G
    Ad = to_device(W.gaussian(100, 40, 5))
    for bad in ((O.BL1, 2), (O.SL1, 41), (O.SL1, 0)):
        with pytest.raises(G.GpspcaError) as e:
            gpu.solve_multistart(Ad, bad[0], bad[1], 1.0, max_iter=3)
        assert e.value.code == G.EINVAL
