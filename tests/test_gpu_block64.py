"""Block solves with m = 64 components (the Stiefel manifold S^p_64, Section 2)
over eight passes against the FP64 oracle, with mu_j = 1 and with mu_j = 1/j
(Table 1, block rows: mu_j multiplies the correlation inside the bracket).

The 2000 x 20000 matrix carries 64 planted 200-sparse components (the block
workload's recipe at a fifth of its size), which selects the same kernels as
the full 64-component workload: the matrix-core correlation with four
component groups, the 64 x 64 FP64 eigensolve of the retraction and, where
most columns are active, the dense matrix-core back-projection.

- BL1, mu_j = 1/j, gamma = 0.005 max||a_i||: every component live, 99% of the
  columns active (dense back-projection).
- BL1, mu_j = 1, gamma = 0.05 max||a_i||: 73% of the columns active.
- BL0, mu_j = 1/j, gamma = 0.01 max||a_i||^2: the threshold on |y| grows as j
  sqrt(gamma), so components past the ninth never pass it; the dead ones are
  completed by reading R7 and the status is DEGENERATE.
- BL0, mu_j = 1, gamma = 0.01 max||a_i||^2: sparse supports, all live.
- BL1X (block L1 from its original form), mu_j = 1/j.

Tolerances are the FP32 path's: X, every Z column and the trace within 1e-5
relative, the same pass count, status and dead set, supports equal outside the
FP32 tie band (l0 cases place gamma away from ties at every oracle iterate).
"""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import fp32_round, is_l0, pick_gamma, rel, tie_mask, to_device, x_to_device

pytestmark = pytest.mark.gpu

TOL = 1e-5
P, N, M, ITERS = 2000, 20000, 64, 8
FNAME = {O.BL1: "BL1", O.BL0: "BL0", O.BL1X: "BL1X"}

_CACHE = {}


@pytest.fixture(scope="module", autouse=True)
def _release():
    yield
    _CACHE.clear()


def _problem():
    if not _CACHE:
        A32, _, _ = W.planted_block(P, N, M, 3, k=200)
        A64 = A32.astype(np.float64)
        X0 = fp32_round(O.init(A64, M)[0])
        _CACHE["p"] = (A32, A64, X0, to_device(A32))
    return _CACHE["p"]


CASES = [
    (O.BL1, "inv", 0.005),
    (O.BL1, "one", 0.05),
    (O.BL0, "inv", 0.01),
    (O.BL0, "one", 0.01),
    (O.BL1X, "inv", 0.005),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{FNAME[c[0]]}-mu_{c[1]}-f{c[2]}")
def test_m64_fixed_passes(gpu, case):
    form, muk, frac = case
    print(f"\n[m64] {FNAME[form]} m={M} p={P} n={N} mu={muk} frac={frac}", flush=True)
    A32, A64, X0, Ad = _problem()
    mu = 1.0 / np.arange(1, M + 1) if muk == "inv" else np.ones(M)
    g0 = W.gamma_absolute(A64, is_l0(form), frac)
    gamma = pick_gamma(A64, form, M, mu, X0, g0, iters=ITERS)
    ref = O.solve(A64, form, M, gamma, mu=mu, X0=X0, tol=0.0, max_iter=ITERS)
    res = gpu.solve(Ad, form, M, gamma, mu=list(mu), X0=x_to_device(X0), tol=0.0,
                    max_iter=ITERS)
    live = ref["support"].any(axis=0)
    print(f"  oracle: status {ref['status']}, live components {int(live.sum())}, "
          f"active columns {ref['support'].any(axis=1).mean():.3f}", flush=True)
    assert res.n_iter == ref["n_iter"] and res.status == ref["status"]
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=TOL)
    X = res.X.cpu().numpy().astype(np.float64)
    Z = res.Z.cpu().numpy().astype(np.float64)
    assert rel(X, ref["X"]) <= TOL
    np.testing.assert_allclose(X.T @ X, np.eye(M), atol=2e-6 * np.sqrt(M))
    for j in range(M):
        assert rel(Z[:, j], ref["Z"][:, j]) <= TOL, j
    sup = res.support_mask().cpu().numpy()
    np.testing.assert_array_equal(sup.any(axis=0), live)
    if is_l0(form):
        np.testing.assert_array_equal(sup, ref["support"])
    else:
        ties = tie_mask(A64, ref["X"], form, gamma, mu)
        assert ties.sum() <= max(2, 1e-3 * ties.size)
        np.testing.assert_array_equal(sup[~ties], ref["support"][~ties])
    if form == O.BL0 and muk == "inv":
        # the mu_j = 1/j case must exercise the dead-component completion
        assert ref["status"] == O.DEGENERATE and 0 < live.sum() < M
