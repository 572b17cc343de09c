"""Pins of the oracle's BL1X: the block-L1 row of Table 1 read from its
original form.  For fixed X, the maximum over unit-norm z_j of
mu_j x_j^T A z_j - gamma ||z_j||_1 is ||s_j|| (s_ij the soft-thresholded
correlation), so the objective is F(X) = sum_j ||s_j(X)|| and the ascent
direction is mu_j A s_j / ||s_j||.

What pins it (nothing here re-types the oracle's formulas):
- the original form evaluated with numpy at the oracle's Z equals the oracle's
  F, and no other unit-norm Z does better (Z is the inner maximizer);
- central differences of the oracle's F match <G, E> for the oracle's
  direction G (a missing or doubled normalization fails this);
- at m = 1 every iterate is the single-unit L1 iterate and F is the square
  root of the SL1 objective (one column's polar factor is its normalization);
- the objective never decreases (power method on a convex function);
- at convergence X is the polar factor of A Z N, computed here by an SVD;
- for m > 1 it differs from the squared reading after one step."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W


def _problem(p, n, m, seed):
    A32, _, _ = W.planted_block(p, n, m, seed, k=min(30, n // (2 * m)))
    A = A32.astype(np.float64)
    cmax = float(np.sqrt((A * A).sum(axis=0)).max())
    return A, cmax


def _original_form(A, X, Z, mu, gamma):
    # Table 1, block L1, original form: Tr(X^T A Z N) - sum_j gamma sum_i |z_ij|
    return float(np.trace(X.T @ A @ Z @ np.diag(mu)) - gamma * np.abs(Z).sum())


@pytest.mark.parametrize("m,seed", [(2, 1), (4, 2), (6, 3)])
def test_objective_is_the_original_form_at_its_inner_maximizer(m, seed):
    A, cmax = _problem(120, 500, m, seed)
    gamma = 0.1 * cmax
    mu = np.linspace(1.0, 0.7, m)
    rng = np.random.default_rng(seed)
    X = np.linalg.qr(rng.standard_normal((120, m)))[0]
    r = O.solve(A, O.BL1X, m, gamma, mu=mu, X0=X, tol=0.0, max_iter=1)
    Z = r["Z"]
    assert r["trace"][0] > 0.0
    np.testing.assert_allclose(_original_form(A, r["X"], Z, mu, gamma), r["trace"][0],
                               rtol=1e-12)
    # any other unit-norm Z gives at most F (Cauchy-Schwarz on the inner problem)
    for _ in range(20):
        Zr = rng.standard_normal(Z.shape) * (Z != 0) + 1e-3 * rng.standard_normal(Z.shape)
        Zr /= np.linalg.norm(Zr, axis=0, keepdims=True)
        assert _original_form(A, r["X"], Zr, mu, gamma) <= r["trace"][0] * (1 + 1e-12)


@pytest.mark.parametrize("m,seed", [(3, 4), (5, 5)])
def test_direction_is_the_gradient_of_the_objective(m, seed):
    A, cmax = _problem(80, 400, m, seed)
    gamma = 0.08 * cmax
    mu = np.linspace(1.0, 0.6, m)
    rng = np.random.default_rng(10 + seed)
    X = np.linalg.qr(rng.standard_normal((80, m)))[0]
    st = O.step(A, O.BL1X, X, gamma, mu=mu)
    assert (st["nnz"] > 0).all()
    h = 1e-6
    for _ in range(5):
        E = rng.standard_normal(X.shape)
        fp = O.step(A, O.BL1X, X + h * E, gamma, mu=mu)["F"]
        fm = O.step(A, O.BL1X, X - h * E, gamma, mu=mu)["F"]
        fd = (fp - fm) / (2 * h)
        np.testing.assert_allclose(fd, float((st["G"] * E).sum()), rtol=1e-6)
    # the squared reading's direction is not this gradient (it scales column j
    # by ||s_j||)
    sq = O.step(A, O.BL1, X, gamma, mu=mu)
    np.testing.assert_allclose(sq["G"], st["G"] * np.sqrt(st["f"])[None, :], rtol=1e-12)


def test_single_component_is_the_single_unit_iteration():
    A, cmax = _problem(150, 700, 1, 6)
    gamma = 0.05 * cmax
    a = O.solve(A, O.BL1X, 1, gamma, tol=0.0, max_iter=12)
    b = O.solve(A, O.SL1, 1, gamma, tol=0.0, max_iter=12)
    assert a["n_iter"] == b["n_iter"]
    np.testing.assert_allclose(a["trace"] ** 2, b["trace"], rtol=1e-12)
    np.testing.assert_allclose(a["X"], b["X"], rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("m,seed", [(3, 7), (8, 8)])
def test_ascent_and_fixed_point(m, seed):
    A, cmax = _problem(100, 600, m, seed)
    gamma = 0.05 * cmax
    mu = np.linspace(1.0, 0.5, m)
    r = O.solve(A, O.BL1X, m, gamma, mu=mu, tol=1e-13, max_iter=3000)
    tr = r["trace"]
    assert r["status"] == O.OK
    assert np.all(np.diff(tr) >= -1e-12 * tr[1:])
    # X is (nearly) the polar factor of A Z N at the end
    U, _, Vt = np.linalg.svd(A @ r["Z"] @ np.diag(mu), full_matrices=False)
    np.testing.assert_allclose(r["X"], U @ Vt, atol=1e-5)


def test_differs_from_the_squared_reading_for_several_components():
    A, cmax = _problem(100, 600, 4, 9)
    gamma = 0.05 * cmax
    mu = np.linspace(1.0, 0.5, 4)
    X0 = O.init(A, 4)[0]
    a = O.solve(A, O.BL1X, 4, gamma, mu=mu, X0=X0, tol=0.0, max_iter=2)
    b = O.solve(A, O.BL1, 4, gamma, mu=mu, X0=X0, tol=0.0, max_iter=2)
    assert np.abs(a["X"] - b["X"]).max() > 1e-4
