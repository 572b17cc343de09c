"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the property it checks.  None of them re-types the oracle's
formulas: they compare against library routines on special cases (SVD,
symmetric eigen-decomposition), closed forms, hand-derived values, brute force
over supports on tiny inputs, and invariances of the Table 1 objectives.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from workloads import generators as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FORMS = [O.SL1, O.SL0, O.BL1, O.BL0]


def _planted_gap(p, n, seed, gap=(9.0, 4.0, 2.0, 1.0)):
    """Tiny A with well separated leading singular values (for the gamma = 0 limits)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((p, p)))
    V, _ = np.linalg.qr(rng.standard_normal((n, p)))
    s = np.linspace(0.5, 0.1, p)
    s[:len(gap)] = gap
    return np.asfortranarray(U @ np.diag(s) @ V.T)


# --- P9: hand-derived p = 1 example (Table 1, t_+ and sign of Section 2) -----

def test_p1_worked_example_golden():
    g = json.load(open(os.path.join(GOLD, "p1_worked_example.json")))
    A = np.array([g["A_row"]])
    for form, key in ((O.SL1, "l1"), (O.SL0, "l0")):
        st = O.step(A, form, np.array([g["x0"]]), g["gamma"])
        np.testing.assert_array_equal(st["S"][:, 0], g[key]["S"])
        assert st["F"] == g[key]["F"]
        x1, _ = O.retract(st["G"], st["nnz"], np.array([[g["x0"]]]))
        assert x1[0, 0] == g[key]["x_next"]
        # negative start keeps its sign
        stn = O.step(A, form, np.array([-g["x0"]]), g["gamma"])
        np.testing.assert_array_equal(stn["S"][:, 0], g["x0_negative"][key + "_S"])
        x1n, _ = O.retract(stn["G"], stn["nnz"], np.array([[-g["x0"]]]))
        assert x1n[0, 0] == g["x0_negative"]["x_next"]
        # original (left-column) form of Table 1 at z = s/||s||
        z = st["S"][:, 0] / np.linalg.norm(st["S"][:, 0])
        Az = float((A @ z)[0])
        orig = (abs(Az) - g["gamma"] * np.abs(z).sum()) if key == "l1" else (Az * Az - g["gamma"] * np.count_nonzero(z))
        assert orig == pytest.approx(g[key]["original_form"], rel=1e-14)


# --- P1 / P2: gamma = 0 reduces to the power method / subspace iteration -----

@pytest.mark.parametrize("form", [O.SL1, O.SL0])
def test_gamma_zero_single_unit_is_power_method(form):
    A = _planted_gap(8, 60, 1)
    U, s, _ = np.linalg.svd(A)
    r = O.solve(A, form, 1, 0.0, tol=0.0, max_iter=400)
    assert abs(r["X"][:, 0] @ U[:, 0]) == pytest.approx(1.0, abs=1e-12)
    assert r["trace"][-1] == pytest.approx(s[0] ** 2, rel=1e-12)


@pytest.mark.parametrize("form", [O.BL1, O.BL0])
def test_gamma_zero_block_distinct_mu_gives_singular_vectors(form):
    A = _planted_gap(10, 80, 2)
    U, s, _ = np.linalg.svd(A)
    mu = np.array([3.0, 2.0, 1.0])
    r = O.solve(A, form, 3, 0.0, mu=mu, tol=0.0, max_iter=3000)
    C = np.abs(r["X"].T @ U[:, :3])
    np.testing.assert_allclose(C, np.eye(3), atol=1e-9)
    assert r["trace"][-1] == pytest.approx(float((mu ** 2 * s[:3] ** 2).sum()), rel=1e-12)


@pytest.mark.parametrize("form", [O.BL1, O.BL0])
def test_gamma_zero_block_unit_mu_gives_subspace(form):
    A = _planted_gap(10, 80, 3)
    U, s, _ = np.linalg.svd(A)
    r = O.solve(A, form, 2, 0.0, tol=0.0, max_iter=2000)
    P = r["X"] @ r["X"].T
    np.testing.assert_allclose(P, U[:, :2] @ U[:, :2].T, atol=1e-9)
    assert r["trace"][-1] == pytest.approx(float((s[:2] ** 2).sum()), rel=1e-12)


# --- P3: large gamma gives the all-zero pattern (Cauchy-Schwarz) ------------

@pytest.mark.parametrize("form", FORMS)
def test_large_gamma_zero_pattern(form):
    A = W.gaussian(12, 50, 4, dtype=np.float64)
    cmax = float(np.sqrt((A ** 2).sum(axis=0)).max())
    m = 1 if form in (O.SL1, O.SL0) else 3
    mu = None if m == 1 else np.array([1.0, 0.5, 0.25])
    mumax = 1.0 if mu is None else mu.max()
    gamma = mumax * cmax if form in (O.SL1, O.BL1) else (mumax * cmax) ** 2
    X0 = W.random_orthonormal(12, m, 5)
    r = O.solve(A, form, m, gamma, mu=mu, X0=X0, tol=1e-6, max_iter=50)
    assert r["n_iter"] == 1
    assert r["status"] == O.DEGENERATE
    assert np.all(r["Z"] == 0.0) and not r["support"].any()
    assert r["trace"][0] == 0.0
    np.testing.assert_allclose(r["X"], O.project(X0), rtol=0, atol=0)
    # just below the bound at least one entry survives for the top column
    if m == 1:
        i = int(np.argmax(np.sqrt((A ** 2).sum(axis=0))))
        x = A[:, i] / np.linalg.norm(A[:, i])
        st = O.step(A, form, x, gamma * (1 - 1e-9))
        assert st["nnz"][0] == 1 and st["S"][i, 0] != 0.0


# --- P4 / P5: monotone objective, feasibility ---------------------------------

@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("frac", [0.02, 0.1, 0.3])
def test_monotone_and_feasible(form, frac):
    A = W.gaussian(30, 200, 7, dtype=np.float64)
    l0 = form in (O.SL0, O.BL0)
    gamma = W.gamma_absolute(A, l0, frac)
    m = 1 if form in (O.SL1, O.SL0) else 4
    mu = None if m == 1 else np.array([1.0, 0.9, 0.8, 0.7])
    r = O.solve(A, form, m, gamma, mu=mu, tol=0.0, max_iter=60)
    tr = r["trace"]
    assert np.all(np.diff(tr) >= -1e-12 * np.abs(tr[1:]))
    X = r["X"]
    np.testing.assert_allclose(X.T @ X, np.eye(m), atol=1e-12)
    nz = np.linalg.norm(r["Z"], axis=0)
    for j in range(m):
        assert nz[j] == pytest.approx(1.0, abs=1e-12) or nz[j] == 0.0


# --- P6: at a fixed point X^T G is symmetric positive semidefinite -----------

@pytest.mark.parametrize("form", [O.BL1, O.BL0])
def test_polar_fixed_point_symmetric_psd(form):
    A = W.gaussian(20, 150, 8, dtype=np.float64)
    gamma = W.gamma_absolute(A, form == O.BL0, 0.05)
    r = O.solve(A, form, 3, gamma, mu=[1.0, 0.8, 0.6], tol=0.0, max_iter=800)
    st = O.step(A, form, r["X"], gamma, mu=[1.0, 0.8, 0.6])
    M = r["X"].T @ st["G"]
    np.testing.assert_allclose(M, M.T, atol=1e-9 * np.abs(M).max())
    assert np.linalg.eigvalsh((M + M.T) / 2).min() >= -1e-9 * np.abs(M).max()


# --- P7: exhaustive search over supports bounds the L0 objective -------------

def _phi_star_l0(A, gamma):
    n = A.shape[1]
    best = 0.0
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            AS = A[:, S]
            lam = np.linalg.eigvalsh(AS.T @ AS)[-1]
            best = max(best, lam - gamma * k)
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exhaustive_l0_upper_bound_and_fixed_point(seed):
    A = W.gaussian(5, 10, 20 + seed, dtype=np.float64)
    gamma = W.gamma_absolute(A, True, 0.3)
    phi = _phi_star_l0(A, gamma)
    best = 0.0
    for s0 in range(6):
        X0 = W.random_orthonormal(5, 1, 100 + s0)
        r = O.solve(A, O.SL0, 1, gamma, X0=X0, tol=0.0, max_iter=300)
        F = r["trace"][-1]
        assert F <= phi * (1 + 1e-12)
        best = max(best, F)
        # fixed point: x is an eigenvector of A_S A_S^T and F = lambda - gamma |S|
        S = np.flatnonzero(r["support"][:, 0])
        if S.size:
            M = A[:, S] @ A[:, S].T
            x = r["X"][:, 0]
            lam = float(x @ M @ x)
            np.testing.assert_allclose(M @ x, lam * x, atol=1e-9 * lam)
            assert F == pytest.approx(lam - gamma * S.size, rel=1e-10)
    assert best >= 0.5 * phi  # multi-start reaches a good part of the optimum


def test_exhaustive_bl0_bound():
    A = W.gaussian(5, 9, 31, dtype=np.float64)
    gamma = W.gamma_absolute(A, True, 0.2)
    mu = np.array([1.0, 0.7])
    bound = sum(mu[j] ** 2 * _phi_star_l0(A, gamma / mu[j] ** 2) for j in range(2))
    r = O.solve(A, O.BL0, 2, gamma, mu=mu, tol=0.0, max_iter=200)
    assert r["trace"][-1] <= bound * (1 + 1e-12)


# --- P8: the two columns of Table 1 agree at Z = Z(X) ------------------------

@pytest.mark.parametrize("form", FORMS)
def test_table1_original_and_reformulation_agree(form):
    A = W.gaussian(15, 120, 9, dtype=np.float64)
    l0 = form in (O.SL0, O.BL0)
    gamma = W.gamma_absolute(A, l0, 0.08)
    m = 1 if form in (O.SL1, O.SL0) else 3
    mu = np.ones(1) if m == 1 else np.array([1.0, 0.75, 0.5])
    X = O.init(A, m)[0]
    Sigma = A.T @ A
    for _ in range(5):
        st = O.step(A, form, X, gamma, mu=None if m == 1 else mu)
        S = st["S"]
        Z = S / np.where(np.linalg.norm(S, axis=0) > 0, np.linalg.norm(S, axis=0), 1.0)
        if l0:
            tr_form = sum((mu[j] * X[:, j] @ A @ Z[:, j]) ** 2 - gamma * np.count_nonzero(Z[:, j])
                          for j in range(m))
            assert tr_form == pytest.approx(st["F"], rel=1e-11)
        else:
            tr_form = sum(mu[j] * X[:, j] @ A @ Z[:, j] - gamma * np.abs(Z[:, j]).sum() for j in range(m))
            assert tr_form == pytest.approx(float(np.sqrt(st["f"]).sum()), rel=1e-11)
        if m == 1:
            z = Z[:, 0]
            if l0:
                assert z @ Sigma @ z - gamma * np.count_nonzero(z) >= st["F"] * (1 - 1e-12)
            else:
                assert np.sqrt(z @ Sigma @ z) - gamma * np.abs(z).sum() >= np.sqrt(st["F"]) * (1 - 1e-12)
        X, _ = O.retract(st["G"], st["nnz"], X)


@pytest.mark.parametrize("form", [O.SL1, O.SL0])
def test_sigma_form_equality_at_fixed_point(form):
    A = W.gaussian(12, 90, 10, dtype=np.float64)
    l0 = form == O.SL0
    gamma = W.gamma_absolute(A, l0, 0.1)
    r = O.solve(A, form, 1, gamma, tol=0.0, max_iter=500)
    z = r["Z"][:, 0]
    Sigma = A.T @ A
    F = r["trace"][-1]
    if l0:
        assert z @ Sigma @ z - gamma * np.count_nonzero(z) == pytest.approx(F, rel=1e-10)
    else:
        assert np.sqrt(z @ Sigma @ z) - gamma * np.abs(z).sum() == pytest.approx(np.sqrt(F), rel=1e-10)


# --- P10: metamorphic invariances --------------------------------------------

@pytest.mark.parametrize("form", FORMS)
def test_scale_invariance(form):
    A = W.gaussian(10, 70, 11, dtype=np.float64)
    l0 = form in (O.SL0, O.BL0)
    gamma = W.gamma_absolute(A, l0, 0.1)
    m = 1 if form in (O.SL1, O.SL0) else 2
    c = 3.0
    X0 = W.random_orthonormal(10, m, 12)
    r1 = O.solve(A, form, m, gamma, X0=X0, tol=0.0, max_iter=40)
    r2 = O.solve(c * A, form, m, gamma * (c * c if l0 else c), X0=X0, tol=0.0, max_iter=40)
    np.testing.assert_allclose(r2["X"], r1["X"], atol=1e-12)
    np.testing.assert_allclose(r2["Z"], r1["Z"], atol=1e-12)
    np.testing.assert_allclose(r2["trace"], c * c * r1["trace"], rtol=1e-12)


@pytest.mark.parametrize("form", FORMS)
def test_permutation_and_rotation_invariance(form):
    A = W.gaussian(10, 70, 13, dtype=np.float64)
    l0 = form in (O.SL0, O.BL0)
    gamma = W.gamma_absolute(A, l0, 0.12)
    m = 1 if form in (O.SL1, O.SL0) else 2
    X0 = W.random_orthonormal(10, m, 14)
    r1 = O.solve(A, form, m, gamma, X0=X0, tol=0.0, max_iter=30)
    perm = np.random.default_rng(15).permutation(70)
    r2 = O.solve(A[:, perm], form, m, gamma, X0=X0, tol=0.0, max_iter=30)
    np.testing.assert_allclose(r2["Z"], r1["Z"][perm], atol=1e-12)
    np.testing.assert_array_equal(r2["support"], r1["support"][perm])
    np.testing.assert_allclose(r2["X"], r1["X"], atol=1e-12)
    Q = W.random_orthonormal(10, 10, 16)
    r3 = O.solve(Q @ A, form, m, gamma, X0=Q @ X0, tol=0.0, max_iter=30)
    np.testing.assert_allclose(r3["X"], Q @ r1["X"], atol=1e-11)
    np.testing.assert_allclose(r3["Z"], r1["Z"], atol=1e-11)
    np.testing.assert_allclose(r3["trace"], r1["trace"], rtol=1e-11)


@pytest.mark.parametrize("l0", [False, True])
def test_mu_placement_matches_single_unit_with_scaled_gamma(l0):
    """Table 1 puts mu_j inside the bracket: [mu|y| - gamma]_+^2 = mu^2 [|y| - gamma/mu]_+^2
    and [(mu y)^2 - gamma]_+ = mu^2 [y^2 - gamma/mu^2]_+."""
    A = W.gaussian(9, 60, 17, dtype=np.float64)
    gamma = W.gamma_absolute(A, l0, 0.15)
    mu = 0.6
    X0 = W.random_orthonormal(9, 1, 18)
    rb = O.solve(A, O.BL0 if l0 else O.BL1, 1, gamma, mu=[mu], X0=X0, tol=0.0, max_iter=25)
    rs = O.solve(A, O.SL0 if l0 else O.SL1, 1, gamma / (mu * mu if l0 else mu), X0=X0, tol=0.0,
                 max_iter=25)
    np.testing.assert_allclose(rb["X"], rs["X"], atol=1e-12)
    np.testing.assert_allclose(rb["Z"], rs["Z"], atol=1e-12)
    np.testing.assert_allclose(rb["trace"], mu * mu * rs["trace"], rtol=1e-12)


# --- P11: diagonal A, closed form ---------------------------------------------

def test_diagonal_l0_closed_form():
    d = np.array([1.0, -4.0, 2.5, 3.0, 0.5])
    A = np.diag(d)
    gamma = 2.0
    r = O.solve(A, O.SL0, 1, gamma, tol=0.0, max_iter=5)
    k = int(np.argmax(np.abs(d)))
    assert np.count_nonzero(r["support"]) == 1 and r["support"][k, 0]
    assert r["trace"][0] == pytest.approx(d[k] ** 2 - gamma, rel=1e-15)
    assert r["trace"][0] == pytest.approx(_phi_star_l0(A, gamma), rel=1e-12)
    np.testing.assert_allclose(np.abs(r["X"][:, 0]), np.eye(5)[k], atol=0)
    r2 = O.solve(A, O.SL0, 1, d[k] ** 2, tol=0.0, max_iter=5)
    assert r2["trace"][0] == 0.0 and r2["n_iter"] == 1


# --- P12: resume --------------------------------------------------------------

@pytest.mark.parametrize("form", [O.SL1, O.BL0])
def test_resume(form):
    A = W.gaussian(14, 100, 19, dtype=np.float64)
    l0 = form == O.BL0
    gamma = W.gamma_absolute(A, l0, 0.05)
    m = 1 if form == O.SL1 else 3
    full = O.solve(A, form, m, gamma, tol=0.0, max_iter=30)
    a = O.solve(A, form, m, gamma, tol=0.0, max_iter=12)
    b = O.solve(A, form, m, gamma, X0=a["X"], tol=0.0, max_iter=19)
    np.testing.assert_allclose(b["trace"], full["trace"][11:30], rtol=1e-12)
    np.testing.assert_allclose(b["X"], full["X"], atol=1e-11)


# --- Polar factor, top-m and dead components ----------------------------------

def test_polar_matches_svd():
    G = W.gaussian(12, 5, 21, dtype=np.float64)
    X, sv, rd = O.polar(G)
    U, s, Vt = np.linalg.svd(G, full_matrices=False)
    np.testing.assert_allclose(X, U @ Vt, atol=1e-13)
    np.testing.assert_allclose(np.sort(sv)[::-1], s, rtol=1e-13)
    assert not rd
    _, _, rd2 = O.polar(np.column_stack([G[:, 0], G[:, 0]]))
    assert rd2


def test_top_m_ties_to_lower_index():
    c = np.array([1.0, 3.0, 2.0, 3.0, 0.5, 2.0])
    np.testing.assert_array_equal(O.top_m(c, 4), [1, 3, 2, 5])


def test_dead_component_completion_is_feasible_and_monotone():
    A = W.gaussian(12, 80, 22, dtype=np.float64)
    gamma = W.gamma_absolute(A, True, 0.2)
    mu = np.array([1.0, 0.5, 0.05])  # third component can never pass the threshold
    r = O.solve(A, O.BL0, 3, gamma, mu=mu, tol=0.0, max_iter=40)
    assert r["status"] == O.DEGENERATE
    assert not r["support"][:, 2].any()
    np.testing.assert_allclose(r["X"].T @ r["X"], np.eye(3), atol=1e-12)
    assert np.all(np.diff(r["trace"]) >= -1e-12 * r["trace"][1:])


def test_validation():
    A = W.gaussian(4, 10, 23, dtype=np.float64)
    with pytest.raises(O.OracleError):
        O.solve(A, O.SL1, 2, 0.1)  # single-unit needs m = 1
    with pytest.raises(O.OracleError):
        O.solve(A, O.BL1, 5, 0.1)  # m > p
    with pytest.raises(O.OracleError):
        O.solve(A, O.BL1, 2, -1.0)
    with pytest.raises(O.OracleError):
        O.solve(A, O.BL1, 2, 0.1, mu=[1.0, 0.0])
    B = A.copy()
    B[0, 0] = np.nan
    with pytest.raises(O.OracleError):
        O.solve(B, O.SL1, 1, 0.1)
