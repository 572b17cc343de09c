"""Parity at the benchmark's full sizes and launch configuration.

The block workload (A 10000 x 100000 FP32, 8 planted 200-sparse components,
seed 0), its 64-component form (64 planted components, beta_j = 5 sqrt(n)/j)
and the single-unit workload (A 5000 x 50000 FP32, one planted 500-sparse
spike) run through the same C-ABI calls and kernel selection as the
benchmark.  The FP64 oracle is fast enough at these sizes to be compared
element by element: one pass (S, G, f, nnz) and three fixed passes of the
solve (X, Z, trace), with supports equal outside the FP32 tie band.

The 32-gamma path runs on the 8-component matrix stored in FP32, bfloat16 and
e4m3 (the oracle's codes and scales), three fixed passes; three of its columns
are compared with the oracle's single-unit solves on the matrix the GPU
reads (the dequantized one for the narrow storage types)."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, TNAME, corr_band, fp32_round, is_l0, pick_gamma, quantized_problem,
                   rel, term_band, tie_mask, to_device, x_to_device)

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
        elif kind == "block64":
            A32, _, _ = W.planted_block(10000, 100000, 64, 0, k=200)
            m = 64
        else:
            A32, _, _, _ = W.planted_single(5000, 50000, 0, k=500)
            m = 1
        A64 = A32.astype(np.float64)
        X0 = fp32_round(O.init(A64, m)[0])
        _CACHE[kind] = (A32, A64, X0, to_device(A32))
    return _CACHE[kind]


def _check_step(gpu, A64, Ad, X0, form, gamma, mu=None):
    m = X0.shape[1]
    ref = O.step(A64, form, X0, gamma, mu=mu)
    out = gpu.step(Ad, form, x_to_device(X0), gamma, mu=None if mu is None else list(mu))
    S = out.S.cpu().numpy().astype(np.float64)
    ties = tie_mask(A64, X0, form, gamma, mu)
    print(f"  step: F={ref['F']:.6g} nnz={list(ref['nnz'])} ties={int(ties.sum())}", flush=True)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    assert np.all(np.abs(np.asarray(out.nnz) - ref["nnz"]) <= ties.sum(axis=0))
    eb = corr_band(A64, X0) * (1.0 if mu is None else np.asarray(mu)[None, :])
    assert np.all(np.abs(S - ref["S"]) <= eb + 1e-7 * np.abs(ref["S"]))
    if is_l0(form):
        assert not ties.any()
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    # the objective within 1e-5; each component's term within 1e-5 plus the FP32
    # band of its summands (with mu_j = 1/j a term can be a small difference of
    # large numbers)
    assert abs(sum(out.f) - ref["F"]) <= 1e-5 * ref["F"]
    fb = term_band(A64, X0, ref["S"], form, mu)
    assert np.all(np.abs(np.asarray(out.f) - ref["f"]) <= 1e-5 * np.abs(ref["f"]) + fb + 1e-9)
    assert m == len(out.f)


def _check_passes(gpu, A64, Ad, X0, form, gamma, iters=3, mu=None):
    m = X0.shape[1]
    ref = O.solve(A64, form, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=iters)
    res = gpu.solve(Ad, form, m, gamma, mu=None if mu is None else list(mu),
                    X0=x_to_device(X0), tol=0.0, max_iter=iters)
    assert res.n_iter == ref["n_iter"] and res.status == ref["status"]
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=1e-5)
    assert rel(res.X.cpu().numpy(), ref["X"]) <= 1e-5
    Z = res.Z.cpu().numpy().astype(np.float64)
    for j in range(m):
        assert rel(Z[:, j], ref["Z"][:, j]) <= 1e-5
    ties = tie_mask(A64, ref["X"], form, gamma, mu)
    sup = res.support_mask().cpu().numpy()
    np.testing.assert_array_equal(sup[~ties], ref["support"][~ties])
    np.testing.assert_array_equal(sup.any(axis=0), ref["support"].any(axis=0))
    return ref


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


@pytest.mark.parametrize("form,muk,frac", [(O.BL1, "one", 0.05), (O.BL1, "inv", 0.005),
                                           (O.BL0, "inv", 0.01)],
                         ids=["BL1-mu1-0.05", "BL1-mu_inv-0.005-dense", "BL0-mu_inv-0.01-dead"])
def test_block_10k_x_100k_m64(gpu, form, muk, frac):
    """64 components on the 64-component matrix: mu_j = 1 at the block L1
    gamma, mu_j = 1/j with most columns active (dense back-projection), and
    BL0 with mu_j = 1/j, where components past the ninth are dead."""
    print(f"\n[fullsize] {FORM_NAMES[form]} m=64 p=10000 n=100000 mu={muk} frac={frac}",
          flush=True)
    A32, A64, X0, Ad = _workload("block64")
    mu = 1.0 / np.arange(1, 65) if muk == "inv" else None
    g0 = W.gamma_absolute(A64, is_l0(form), frac)
    gamma = pick_gamma(A64, form, 64, mu, X0, g0, iters=3)
    _check_step(gpu, A64, Ad, X0, form, gamma, mu=mu)
    ref = _check_passes(gpu, A64, Ad, X0, form, gamma, mu=mu)
    if form == O.BL0:
        live = int(ref["support"].any(axis=0).sum())
        print(f"  live components {live} of 64, status {ref['status']}", flush=True)
        assert ref["status"] == O.DEGENERATE and 0 < live < 64


@pytest.mark.parametrize("form", [O.SL1, O.SL0], ids=["SL1", "SL0"])
@pytest.mark.parametrize("to", ["f32", O.BF16, O.E4M3], ids=["f32", "bf16", "e4m3"])
def test_gamma_path_10k_x_100k_k32(gpu, to, form):
    """32 gammas, log-spaced fractions 0.01 .. 0.5, from the largest-norm
    column, three fixed passes; columns 0, 15 and 31 against the oracle."""
    import torch
    print(f"\n[fullsize] path K=32 {FORM_NAMES[form]} storage={TNAME.get(to, 'f32')}",
          flush=True)
    A32, A64, _, Ad = _workload("block")
    sc = None
    if to != "f32":
        A32q, Aref, Ad, sc = quantized_problem(10000, 100000, 1, 0, to, A32=A32)
    else:
        Aref = A64
    x0 = fp32_round(O.init(Aref, 1)[0])
    K, iters = 32, 3
    gammas = [W.gamma_absolute(Aref, is_l0(form), f) for f in W.gamma_fractions(K)]
    sample = (0, 15, 31)
    for k in sample:
        gammas[k] = pick_gamma(Aref, form, 1, None, x0, gammas[k], iters=iters)
    res = gpu.solve_path(Ad, form, gammas, X0=x_to_device(np.repeat(x0, K, axis=1)), tol=0.0,
                         max_iter=iters, col_scale=sc)
    X = res.X.cpu().numpy().astype(np.float64)
    Z = res.Z.cpu().numpy().astype(np.float64)
    sup = res.support_mask().cpu().numpy()
    for k in sample:
        ref = O.solve(Aref, form, 1, gammas[k], X0=x0, tol=0.0, max_iter=iters)
        assert res.n_iter[k] == ref["n_iter"] and res.status[k] == ref["status"], k
        np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
        assert rel(X[:, k], ref["X"][:, 0]) <= 1e-5, k
        assert rel(Z[:, k], ref["Z"][:, 0]) <= 1e-5, k
        ties = tie_mask(Aref, ref["X"], form, gammas[k], None)[:, 0]
        print(f"  column {k}: F={ref['trace'][-1]:.6g} nnz={int(ref['support'].sum())} "
              f"ties={int(ties.sum())}", flush=True)
        np.testing.assert_array_equal(sup[~ties, k], ref["support"][~ties, 0])
    del Ad, sc
    torch.cuda.empty_cache()
