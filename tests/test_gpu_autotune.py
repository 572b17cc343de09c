"""The autotuner: it times the candidate configurations, records the fastest,
and later solves (which then run the tuned configuration) still match the FP64
oracle; clearing the table restores the defaults."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import generators as W

from _util import fp32_round, is_l0, pick_gamma, rel, to_device, x_to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clear(gpu):
    gpu.autotune_clear()
    yield
    gpu.autotune_clear()


@pytest.mark.parametrize("form,m,store", [(O.BL1, 8, "f32"), (O.BL0, 20, "f32"),
                                          (O.SL1, 8, "f32"), (O.BL1, 4, "bf16")])
def test_tuned_solves_match_the_oracle(gpu, form, m, store):
    p, n, iters = 1200, 6000, 8
    A32, _, _ = W.planted_block(p, n, min(m, 4), 3 + m, k=40)
    Ad = to_device(A32)
    sc = None
    if store == "bf16":
        Ad, sc = gpu.quantize(Ad, torch.bfloat16)
        codes = Ad.t().contiguous().cpu().view(torch.int16).numpy().view(np.uint16).T
        A64 = O.dequantize(np.asfortranarray(codes), O.BF16, None, p)
    else:
        A64 = A32.astype(np.float64)
    single = form in (O.SL1, O.SL0)
    X0 = fp32_round(O.init(A64, 1 if single else m)[0])
    g = W.gamma_absolute(A64, is_l0(form), 0.05)
    if single:
        X0 = np.repeat(X0, m, axis=1)        # a gamma path of m equal problems
    rep = gpu.autotune(Ad, form, m, g, X0=x_to_device(X0), passes=2, col_scale=sc)
    print(f"\n[autotune] {form} m={m} {store}: {rep}", flush=True)
    assert rep["timed"] >= 2 and rep["best_ms_per_pass"] > 0 and rep["choice"]
    if single:
        res = gpu.solve_path(Ad, form, [g] * m, X0=x_to_device(X0), tol=0.0, max_iter=iters,
                             col_scale=sc)
        ref = O.solve(A64, form, 1, g, X0=X0[:, :1], tol=0.0, max_iter=iters)
        for k in (0, m - 1):
            np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
            assert rel(res.X[:, k].cpu().numpy(), ref["X"][:, 0]) <= 1e-5
    else:
        g = pick_gamma(A64, form, m, None, X0, g, iters=iters)
        res = gpu.solve(Ad, form, m, g, X0=x_to_device(X0), tol=0.0, max_iter=iters, col_scale=sc)
        ref = O.solve(A64, form, m, g, X0=X0, tol=0.0, max_iter=iters)
        np.testing.assert_allclose(res.trace, ref["trace"], rtol=1e-5)
        assert rel(res.X.cpu().numpy(), ref["X"]) <= 1e-5


def test_tuned_configuration_is_deterministic_and_clearable(gpu):
    A32, _, _ = W.planted_block(1000, 8000, 4, 9, k=40)
    Ad = to_device(A32)
    g = W.gamma_absolute(A32.astype(np.float64), False, 0.05)
    base = gpu.solve(Ad, O.BL1, 8, g, tol=0.0, max_iter=6)
    gpu.autotune(Ad, O.BL1, 8, g, passes=2)
    a = gpu.solve(Ad, O.BL1, 8, g, tol=0.0, max_iter=6)
    b = gpu.solve(Ad, O.BL1, 8, g, tol=0.0, max_iter=6)
    np.testing.assert_array_equal(a.X.cpu().numpy(), b.X.cpu().numpy())
    assert rel(a.X.cpu().numpy(), base.X.cpu().numpy()) <= 1e-5
    gpu.autotune_clear()
    c = gpu.solve(Ad, O.BL1, 8, g, tol=0.0, max_iter=6)
    np.testing.assert_array_equal(c.X.cpu().numpy(), base.X.cpu().numpy())
