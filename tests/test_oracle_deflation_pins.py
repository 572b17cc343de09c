"""Pins of the oracle's deflated single-unit components (oracle.solve_deflated,
a reading of the paper's single-unit runs with several components, Section
4.1): closed forms and invariants that do not come from the oracle itself."""
import numpy as np
import pytest

import oracle as O


def _gapped(p, n, sv, seed):
    """A = U diag(sv) V^T with the given singular values (clear gaps)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((p, len(sv))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(sv))))
    return np.asfortranarray((U * np.asarray(sv)) @ V.T), U


@pytest.mark.parametrize("form", [O.SL1, O.SL0])
def test_gamma_zero_gives_the_leading_singular_vectors_in_order(form):
    # gamma = 0: each deflated single-unit solve is the power method on A_k A_k^T,
    # whose top eigenvector is the next left singular vector of A
    A, U = _gapped(40, 200, [9.0, 6.0, 4.0, 2.5, 1.0], 3)
    r = O.solve_deflated(A, form, 3, 0.0, tol=0.0, max_iter=400)
    for k in range(3):
        assert abs(float(U[:, k] @ r["X"][:, k])) > 1 - 1e-10
        # F = sigma_k^2 (the objective of the power method at its fixed point)
        assert r["traces"][k][-1] == pytest.approx([81.0, 36.0, 16.0][k], rel=1e-9)


@pytest.mark.parametrize("form,frac", [(O.SL1, 0.05), (O.SL0, 0.005)])
def test_components_are_orthonormal_and_the_first_is_the_plain_solve(form, frac):
    rng = np.random.default_rng(11)
    A = np.asfortranarray(rng.standard_normal((60, 400)))
    c = np.sqrt((A ** 2).sum(axis=0)).max()
    g = frac * (c * c if form == O.SL0 else c)
    r = O.solve_deflated(A, form, 4, g, tol=1e-10, max_iter=300)
    X = r["X"]
    np.testing.assert_allclose(X.T @ X, np.eye(4), atol=1e-10)
    plain = O.solve(A, form, 1, g, tol=1e-10, max_iter=300)
    np.testing.assert_array_equal(X[:, 0], plain["X"][:, 0])
    assert r["n_iter"][0] == plain["n_iter"]


def test_components_start_at_the_largest_deflated_column():
    # with a single pass a solve returns its start (the iterate X_0 of that
    # pass): component 1 starts at the normalized largest-norm column of A,
    # component 2 at the normalized largest column of A_1 = (I - x1 x1^T) A
    rng = np.random.default_rng(5)
    A = np.asfortranarray(rng.standard_normal((30, 100)))
    c0 = np.sqrt((A ** 2).sum(axis=0))
    i1 = int(np.argmax(c0))
    x1 = A[:, i1] / c0[i1]
    A1 = A - np.outer(x1, x1 @ A)
    c1 = np.sqrt((A1 ** 2).sum(axis=0))
    i2 = int(np.argmax(c1))
    r = O.solve_deflated(A, O.SL1, 2, 0.1 * c0.max(), tol=0.0, max_iter=1)
    np.testing.assert_allclose(r["X"][:, 0], x1, atol=1e-13)
    np.testing.assert_allclose(r["X"][:, 1], A1[:, i2] / c1[i2], atol=1e-12)
    assert r["n_iter"] == [1, 1]
