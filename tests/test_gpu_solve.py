"""Solve parity: full power iterations of the HIP path (gpspca_solve through the
C ABI) against the FP64 oracle from the same start, with tol = 0 and a fixed
pass count so both stop at the same k.  X, Z and the objective trace within
1e-5 relative; supports exactly equal outside the FP32 tie band (l0 cases place
gamma away from ties at every oracle iterate)."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, fp32_round, is_l0, pick_gamma, rel, tie_mask, to_device,
                   x_to_device)

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _compare(res, ref, m, A64=None, form=None, gamma=None, mu=None):
    """Supports compared outside the FP32 tie band of the final iterate (l1 forms
    only; l0 cases place gamma away from ties at every iterate)."""
    X = res.X.cpu().numpy().astype(np.float64)
    Z = res.Z.cpu().numpy().astype(np.float64)
    assert res.n_iter == ref["n_iter"]
    assert res.status == ref["status"]
    sup = res.support_mask().cpu().numpy()
    if A64 is not None and not is_l0(form):
        ties = tie_mask(A64, ref["X"], form, gamma, mu)
        assert ties.sum() <= max(2, 1e-3 * ties.size)
        np.testing.assert_array_equal(sup[~ties], ref["support"][~ties])
    else:
        np.testing.assert_array_equal(sup, ref["support"])
    assert rel(X, ref["X"]) <= TOL
    for j in range(m):
        assert rel(Z[:, j], ref["Z"][:, j]) <= TOL
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=TOL)


CASES = [
    (O.SL1, 1, 700, 4001, 1),
    (O.SL0, 1, 700, 4001, 2),
    (O.SL1, 1, 3001, 2500, 3),
    (O.SL0, 1, 257, 9000, 4),
    (O.BL1, 4, 600, 3000, 5),
    (O.BL0, 4, 600, 3000, 6),
    (O.BL1, 8, 1500, 2500, 7),
    (O.BL0, 8, 1500, 2500, 8),
    (O.BL1, 16, 400, 2000, 9),
    (O.BL0, 12, 400, 2000, 10),
]


@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"{FORM_NAMES[c[0]]}-m{c[1]}-p{c[2]}-n{c[3]}")
def test_solve_parity_fixed_passes(gpu, case):
    form, m, p, n, seed = case
    iters = 12
    print(f"\n[solve] {FORM_NAMES[form]} m={m} p={p} n={n} seed={seed}", flush=True)
    A32, _, _ = W.planted_block(p, n, min(m, 4), seed, k=40)
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.8, m) if form >= O.BL1 else None
    X0 = fp32_round(O.init(A64, m)[0])
    g0 = W.gamma_absolute(A64, is_l0(form), 0.03 if is_l0(form) else 0.06)
    gamma = pick_gamma(A64, form, m, mu, X0, g0, iters=iters)
    ref = O.solve(A64, form, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=iters)
    res = gpu.solve(to_device(A32), form, m, gamma, mu=None if mu is None else list(mu),
                    X0=x_to_device(X0), tol=0.0, max_iter=iters)
    _compare(res, ref, m, A64, form, gamma, mu)


@pytest.mark.parametrize("form", [O.SL1, O.BL0])
def test_default_start_matches_oracle(gpu, form):
    """X0 = NULL: top-m norm columns (separated norms) then projection."""
    p, n = 300, 2000
    m = 1 if form == O.SL1 else 5
    A32 = W.gaussian(p, n, 31)
    scale = np.ones(n, dtype=np.float32)
    cols = np.random.default_rng(32).choice(n, size=m, replace=False)
    scale[cols] = 1.5 + 0.1 * np.arange(m)
    A32 = np.asfortranarray(A32 * scale[None, :])
    A64 = A32.astype(np.float64)
    Xi, idx = O.init(A64, m)
    assert set(idx) == set(cols)
    g0 = W.gamma_absolute(A64, is_l0(form), 0.05)
    gamma = pick_gamma(A64, form, m, None, Xi, g0, iters=6)
    ref = O.solve(A64, form, m, gamma, tol=0.0, max_iter=6)
    res = gpu.solve(to_device(A32), form, m, gamma, tol=0.0, max_iter=6)
    _compare(res, ref, m, A64, form, gamma, None)


def test_paper_shape_c1_converged(gpu):
    """100 x 1000 centred Gaussian, SL1, gamma = 0.1 max ||a_i||, default start,
    tol 1e-4, up to 1000 passes: same stopping pass and result as the oracle."""
    A64 = W.gaussian_centered(100, 1000, 0)
    A32 = np.asfortranarray(A64.astype(np.float32))
    A64 = A32.astype(np.float64)
    g0 = W.gamma_absolute(A64, False, 0.1)
    X0 = O.init(A64, 1)[0]
    gamma = pick_gamma(A64, O.SL1, 1, None, X0, g0, iters=40)
    ref = O.solve(A64, O.SL1, 1, gamma, tol=1e-4, max_iter=1000)
    tr = ref["trace"]
    # the tolerance decision is far from its threshold on both sides
    ratios = np.abs(np.diff(tr)) / np.abs(tr[:-1])
    assert np.all(np.abs(ratios - 1e-4) > 1e-6)
    res = gpu.solve(to_device(A32), O.SL1, 1, gamma, tol=1e-4, max_iter=1000)
    _compare(res, ref, 1, A64, O.SL1, gamma, None)


@pytest.mark.parametrize("form", [O.SL1, O.SL0, O.BL1, O.BL0])
def test_large_gamma_zero_pattern(gpu, form):
    p, n = 64, 500
    m = 1 if form < O.BL1 else 3
    A32 = W.gaussian(p, n, 41)
    A64 = A32.astype(np.float64)
    cmax = np.sqrt((A64 ** 2).sum(axis=0)).max()
    gamma = 1.01 * (cmax ** 2 if is_l0(form) else cmax)
    X0 = fp32_round(W.random_orthonormal(p, m, 42))
    res = gpu.solve(to_device(A32), form, m, gamma, X0=x_to_device(X0), tol=1e-4, max_iter=50)
    assert res.n_iter == 1 and res.status == O.DEGENERATE
    assert res.trace == [0.0]
    assert float(res.Z.abs().max()) == 0.0
    assert int(res.support.abs().sum()) == 0
    assert rel(res.X.cpu().numpy(), O.project(X0)) <= 1e-6


def test_dead_component_completion(gpu):
    """BL0 with a component weight too small to pass the threshold: the dead
    column is completed by the same rule as the oracle."""
    p, n, m = 80, 1200, 3
    A32, _, _ = W.planted_block(p, n, 2, 51, k=30)
    A64 = A32.astype(np.float64)
    mu = np.array([1.0, 0.9, 0.02])
    X0 = fp32_round(O.init(A64, m)[0])
    g0 = W.gamma_absolute(A64, True, 0.05)
    gamma = pick_gamma(A64, O.BL0, m, mu, X0, g0, iters=8)
    ref = O.solve(A64, O.BL0, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=8)
    assert ref["status"] == O.DEGENERATE and not ref["support"][:, 2].any()
    res = gpu.solve(to_device(A32), O.BL0, m, gamma, mu=list(mu), X0=x_to_device(X0), tol=0.0,
                    max_iter=8)
    _compare(res, ref, m)
    X = res.X.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(X.T @ X, np.eye(m), atol=1e-6)


@pytest.mark.parametrize("shape", [(1, 50, 1), (2, 7, 1), (3, 1, 1), (5, 40, 5), (9, 33, 9)])
def test_degenerate_shapes(gpu, shape):
    """p = 1, tiny p (ragged quad only), n = 1, and m = p (square X)."""
    p, n, m = shape
    form = O.SL0 if m == 1 else O.BL1
    A32 = W.gaussian(p, n, 61)
    A64 = A32.astype(np.float64)
    X0 = fp32_round(W.random_orthonormal(p, m, 62)) if p > 1 else np.ones((1, 1))
    g0 = W.gamma_absolute(A64, is_l0(form), 0.1)
    gamma = pick_gamma(A64, form, m, None, X0, g0, iters=5)
    ref = O.solve(A64, form, m, gamma, X0=X0, tol=0.0, max_iter=5)
    res = gpu.solve(to_device(A32), form, m, gamma, X0=x_to_device(X0), tol=0.0, max_iter=5)
    _compare(res, ref, m, A64, form, gamma, None)


def test_deterministic_bitwise(gpu):
    p, n, m = 1200, 6000, 8
    A32, _, _ = W.planted_block(p, n, 4, 71, k=40)
    Ad = to_device(A32)
    g = W.gamma_absolute(A32.astype(np.float64), False, 0.03)
    r1 = gpu.solve(Ad, O.BL1, m, g, tol=0.0, max_iter=10)
    r2 = gpu.solve(Ad, O.BL1, m, g, tol=0.0, max_iter=10)
    assert r1.trace == r2.trace
    assert bool((r1.X == r2.X).all()) and bool((r1.Z == r2.Z).all())


def test_resume_equals_longer_run(gpu):
    p, n = 500, 3000
    A32 = W.gaussian(p, n, 81)
    Ad = to_device(A32)
    g = W.gamma_absolute(A32.astype(np.float64), False, 0.05)
    full = gpu.solve(Ad, O.SL1, 1, g, tol=0.0, max_iter=20)
    a = gpu.solve(Ad, O.SL1, 1, g, tol=0.0, max_iter=8)
    b = gpu.solve(Ad, O.SL1, 1, g, X0=a.X, tol=0.0, max_iter=13)
    np.testing.assert_allclose(b.trace, full.trace[7:20], rtol=1e-6)
    assert rel(b.X.cpu().numpy(), full.X.cpu().numpy()) <= 1e-6


def test_rank_deficient_start_rejected(gpu):
    import paper_1312_6182_amd as G
    p, n = 50, 300
    A32 = W.gaussian(p, n, 91)
    x = np.ones((p, 1))
    X0 = np.hstack([x, x]).astype(np.float32)
    with pytest.raises(G.GpspcaError) as ei:
        gpu.solve(to_device(A32), O.BL1, 2, 0.1, X0=x_to_device(X0), tol=0.0, max_iter=3)
    assert ei.value.code == O.EINVAL
