"""Pins of the oracle's reduced-precision storage and of its frozen-support
(masked) passes, against library conversions, exhaustive code tables and
special cases -- not against the oracle's own formulas."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import generators as W


def _torch_bf16_codes(v):
    return torch.from_numpy(np.asarray(v, np.float32)).to(torch.bfloat16).view(torch.int16) \
        .numpy().astype(np.uint16)


def _torch_e4m3_codes(v):
    return torch.from_numpy(np.asarray(v, np.float32)).to(torch.float8_e4m3fn) \
        .view(torch.uint8).numpy()


def _random_floats(seed, count=200000):
    rng = np.random.default_rng(seed)
    mags = 10.0 ** rng.uniform(-8, 8, count)
    return (rng.choice([-1.0, 1.0], count) * mags * rng.uniform(0.5, 1.0, count)).astype(np.float32)


def test_bf16_matches_torch_rounding():
    v = np.concatenate([_random_floats(1), np.float32(1e-39) * _random_floats(2, 5000) / 1e8,
                        np.array([0.0, -0.0, 3.0e38, -3.0e38, 1.0, -1.0], np.float32)])
    np.testing.assert_array_equal(O.encode(v, O.BF16), _torch_bf16_codes(v))


def test_bf16_ties_go_to_even():
    # midpoints between consecutive bfloat16 values are exact FP32 numbers
    codes = np.arange(0x3F80, 0x3F80 + 256, dtype=np.uint16)
    lo = O.decode(codes[:-1], O.BF16)
    hi = O.decode(codes[1:], O.BF16)
    mid = ((lo + hi) / 2).astype(np.float32)
    got = O.encode(mid, O.BF16)
    even = np.where(codes[:-1] % 2 == 0, codes[:-1], codes[1:])
    np.testing.assert_array_equal(got, even)


def test_bf16_code_table_round_trip():
    codes = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    vals = O.decode(codes, O.BF16)
    finite = np.isfinite(vals)
    np.testing.assert_array_equal(O.encode(vals[finite].astype(np.float32), O.BF16), codes[finite])
    ref = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(vals[finite], ref[finite].astype(np.float64))


def test_e4m3_matches_torch_rounding_in_range():
    v = _random_floats(3)
    v = v[np.abs(v) <= 448.0]
    v = np.concatenate([v, np.array([0.0, -0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 2.0 ** -6,
                                     0.0019, 1e-4, 464.0 - 1e-3], np.float32)])
    v = v[np.abs(v) <= 448.0]
    np.testing.assert_array_equal(O.encode(v, O.E4M3), _torch_e4m3_codes(v))


def test_e4m3_code_table():
    codes = np.arange(256, dtype=np.uint16).astype(np.uint8)
    finite = (codes & 0x7F) != 0x7F          # 0x7F and 0xFF are NaN in e4m3fn
    vals = O.decode(codes, O.E4M3)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    np.testing.assert_array_equal(vals[finite], ref[finite])
    np.testing.assert_array_equal(O.encode(vals[finite].astype(np.float32), O.E4M3), codes[finite])
    assert vals[0x7E] == 448.0 and vals[0x08] == 2.0 ** -6 and vals[0x01] == 2.0 ** -9


def test_e4m3_ties_and_saturation():
    codes = np.arange(0x00, 0x7E, dtype=np.uint8)
    lo, hi = O.decode(codes, O.E4M3), O.decode(codes + 1, O.E4M3)
    mid = ((lo + hi) / 2).astype(np.float32)
    even = np.where(codes % 2 == 0, codes, codes + 1).astype(np.uint8)
    np.testing.assert_array_equal(O.encode(mid, O.E4M3), even)
    big = np.array([448.0, 449.0, 464.0, 500.0, 1e6, 3e38], np.float32)
    np.testing.assert_array_equal(O.encode(big, O.E4M3), np.full(6, 0x7E, np.uint8))
    np.testing.assert_array_equal(O.encode(-big, O.E4M3), np.full(6, 0xFE, np.uint8))


@pytest.mark.parametrize("to", [O.BF16, O.E4M3])
def test_quantize_columns(to):
    A = W.gaussian(37, 300, 5)
    A[:, 7] = 0.0                                    # a zero column
    A[:, 8] *= 1e-3
    codes, scale = O.quantize(A, to, ldq=48)
    D = O.dequantize(codes, to, scale, 37)
    amax = np.abs(A).max(axis=0).astype(np.float32)
    if to == O.BF16:
        np.testing.assert_array_equal(scale, np.ones(300, np.float32))
        assert np.all(np.abs(D - A) <= 2.0 ** -8 * np.abs(A.astype(np.float64)))
        np.testing.assert_array_equal(codes[:37], _torch_bf16_codes(A))
    else:
        expect = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
        np.testing.assert_array_equal(scale, expect)
        # the largest entry of every non-zero column maps to +-448
        i = np.abs(A).argmax(axis=0)
        top = codes[i, np.arange(300)]
        assert np.all((top[amax > 0] & 0x7F) == 0x7E)
        ref = _torch_e4m3_codes(A / scale[None, :])
        np.testing.assert_array_equal(codes[:37], ref)
        # half-ulp bound in the normal range, half the subnormal spacing below
        rel_bound = 2.0 ** -4 * np.abs(A.astype(np.float64)) + 2.0 ** -10 * scale[None, :]
        assert np.all(np.abs(D - A) <= rel_bound)
        assert np.all(D[:, 7] == 0.0)


def test_mask_of_ones_is_the_plain_pass():
    A = W.gaussian(40, 300, 6).astype(np.float64)
    X = O.init(A, 3)[0]
    g = W.gamma_absolute(A, False, 0.1)
    a = O.step(A, O.BL1, X, g)
    b = O.step(A, O.BL1, X, g, mask=np.ones((300, 3), bool))
    for k in ("S", "G", "f", "nnz"):
        np.testing.assert_array_equal(a[k], b[k])


def test_column_mask_equals_pass_on_column_subset():
    A = W.gaussian(30, 400, 7).astype(np.float64)
    X = O.init(A, 1)[0]
    g = W.gamma_absolute(A, True, 0.002)
    keep = np.zeros(400, bool)
    keep[np.random.default_rng(8).choice(400, 150, replace=False)] = True
    full = O.step(A, O.SL0, X, g, mask=keep[:, None])
    sub = O.step(A[:, keep], O.SL0, X, g)
    np.testing.assert_allclose(full["G"], sub["G"], rtol=1e-13, atol=1e-13)
    assert full["nnz"][0] == sub["nnz"][0]
    np.testing.assert_allclose(full["F"], sub["F"], rtol=1e-13)
    assert np.all(full["S"][~keep] == 0.0)


@pytest.mark.parametrize("form", [O.SL1, O.BL0])
def test_mask_at_converged_support_keeps_the_fixed_point(form):
    A32, _, _ = W.planted_block(60, 800, 2, 9, k=40)
    A = A32.astype(np.float64)
    m = 1 if form == O.SL1 else 2
    g = W.gamma_absolute(A, form == O.BL0, 0.2 if form == O.SL1 else 0.05)
    ref = O.solve(A, form, m, g, tol=0.0, max_iter=300)
    again = O.solve(A, form, m, g, X0=ref["X"], tol=0.0, max_iter=3, mask=ref["support"])
    np.testing.assert_array_equal(again["support"], ref["support"])
    np.testing.assert_allclose(again["X"], ref["X"], atol=1e-9)
    np.testing.assert_allclose(again["trace"][-1], ref["trace"][-1], rtol=1e-10)
