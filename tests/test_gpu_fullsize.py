"""Parity at the benchmark's full sizes and launch configuration.

The block workload (A 10000 x 100000 FP32, 8 planted 200-sparse components,
seed 0) and the single-unit workload (A 5000 x 50000 FP32, one planted
500-sparse spike) run through the same C-ABI calls and kernel selection as the
benchmark.  The FP64 oracle is fast enough at these sizes to be compared
element by element: one pass (S, G, f, nnz) and three fixed passes of the
solve (X, Z, trace), with supports equal outside the FP32 tie band."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, corr_band, fp32_round, is_l0, pick_gamma, rel, tie_mask,
                   to_device, x_to_device)

pytestmark = pytest.mark.gpu

_CACHE = {}


@pytest.fixture(scope="module", autouse=True)
def _release():
    yield
    _CACHE.clear()


def _workload(kind):
    """(A32, A64, X0) of the block (10k x 100k) or single-unit (5k x 50k) workload."""
    if kind not in _CACHE:
        _CACHE.clear()
        if kind == "block":
            A32, _, _ = W.planted_block(10000, 100000, 8, 0, k=200)
            m = 8
        else:
            A32, _, _, _ = W.planted_single(5000, 50000, 0, k=500)
            m = 1
        A64 = A32.astype(np.float64)
        X0 = fp32_round(O.init(A64, m)[0])
        _CACHE[kind] = (A32, A64, X0, to_device(A32))
    return _CACHE[kind]


def _check_step(gpu, A64, Ad, X0, form, gamma):
    m = X0.shape[1]
    ref = O.step(A64, form, X0, gamma)
    out = gpu.step(Ad, form, x_to_device(X0), gamma)
    S = out.S.cpu().numpy().astype(np.float64)
    ties = tie_mask(A64, X0, form, gamma, None)
    print(f"  step: F={ref['F']:.6g} nnz={list(ref['nnz'])} ties={int(ties.sum())}", flush=True)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    assert np.all(np.abs(np.asarray(out.nnz) - ref["nnz"]) <= ties.sum(axis=0))
    eb = corr_band(A64, X0)
    assert np.all(np.abs(S - ref["S"]) <= eb + 1e-7 * np.abs(ref["S"]))
    if is_l0(form):
        assert not ties.any()
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5, atol=1e-9 * max(1.0, ref["F"]))
    assert m == len(out.f)


def _check_passes(gpu, A64, Ad, X0, form, gamma, iters=3):
    m = X0.shape[1]
    ref = O.solve(A64, form, m, gamma, X0=X0, tol=0.0, max_iter=iters)
    res = gpu.solve(Ad, form, m, gamma, X0=x_to_device(X0), tol=0.0, max_iter=iters)
    assert res.n_iter == ref["n_iter"] and res.status == ref["status"]
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=1e-5)
    assert rel(res.X.cpu().numpy(), ref["X"]) <= 1e-5
    Z = res.Z.cpu().numpy().astype(np.float64)
    for j in range(m):
        assert rel(Z[:, j], ref["Z"][:, j]) <= 1e-5
    ties = tie_mask(A64, ref["X"], form, gamma, None)
    sup = res.support_mask().cpu().numpy()
    np.testing.assert_array_equal(sup[~ties], ref["support"][~ties])


@pytest.mark.parametrize("form,frac", [(O.BL1, 0.05), (O.BL0, 0.01)],
                         ids=lambda v: FORM_NAMES.get(v, str(v)) if isinstance(v, int) else str(v))
def test_block_10k_x_100k_m8(gpu, form, frac):
    print(f"\n[fullsize] {FORM_NAMES[form]} m=8 p=10000 n=100000 frac={frac}", flush=True)
    A32, A64, X0, Ad = _workload("block")
    g0 = W.gamma_absolute(A64, is_l0(form), frac)
    gamma = pick_gamma(A64, form, 8, None, X0, g0, iters=3)
    _check_step(gpu, A64, Ad, X0, form, gamma)
    _check_passes(gpu, A64, Ad, X0, form, gamma)


@pytest.mark.parametrize("form,frac", [(O.SL1, 0.05), (O.SL0, 0.01), (O.SL1, 0.01)],
                         ids=["SL1-0.05", "SL0-0.01", "SL1-0.01-dense"])
def test_single_unit_5k_x_50k(gpu, form, frac):
    print(f"\n[fullsize] {FORM_NAMES[form]} m=1 p=5000 n=50000 frac={frac}", flush=True)
    A32, A64, X0, Ad = _workload("single")
    g0 = W.gamma_absolute(A64, is_l0(form), frac)
    gamma = pick_gamma(A64, form, 1, None, X0, g0, iters=3)
    _check_step(gpu, A64, Ad, X0, form, gamma)
    _check_passes(gpu, A64, Ad, X0, form, gamma)
