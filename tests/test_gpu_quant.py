"""Reduced-precision storage on the GPU (bfloat16 and e4m3fn with per-column
scales) against the FP64 oracle.

- gpspca_quantize: codes and scales bit-exact against the oracle's quantizer.
- Passes and solves on quantized A: against the oracle run on the dequantized
  matrix (scale_i * value(q_ri), exact in FP64), to the same tolerances as the
  FP32 path (supports exact outside the tie band, S within the band, G, X, Z
  and the objective within 1e-5 relative).  The quantized matrices are the
  oracle's codes; the GPU quantizer is only checked against them.
- Refinement on a frozen support: GPU passes on FP32 A started from the
  oracle's reduced-precision result and support, against the oracle's masked
  solve from the same inputs.
"""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, TD, TNAME, corr_band, fp32_round, is_l0, pick_gamma,
                   quantized_problem, rel, tie_mask, to_device, x_to_device)

pytestmark = pytest.mark.gpu

def _words_to_device(mask):
    """(n, m) bool -> (m, ceil(n/32)) int32 words."""
    n, m = mask.shape
    nw = (n + 31) // 32
    bits = np.zeros((m, nw * 32), dtype=np.uint64)
    bits[:, :n] = mask.T
    w = (bits.reshape(m, nw, 32) << np.arange(32, dtype=np.uint64)).sum(axis=2)
    return torch.from_numpy(w.astype(np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
def test_quantize_bit_exact(gpu, to):
    rng = np.random.default_rng(3)
    p, n = 1003, 777
    A = W.gaussian(p, n, 4)
    A[:, 5] = 0.0
    A[:, 6] *= 1e-30
    A[:, 7] *= 1e6
    A[:17, 8] = rng.choice([-1.0, 1.0], 17) * (2.0 ** -9) * 448 * rng.integers(1, 9, 17)
    ldq = 1008
    ref_codes, ref_scale = O.quantize(A, to, ldq=ldq)
    Aq, sc = gpu.quantize(to_device(A), TD[to])
    assert Aq.stride(1) == ldq
    got = Aq.t().contiguous().cpu()
    got = (got.view(torch.int16).numpy().view(np.uint16) if to == O.BF16
           else got.view(torch.uint8).numpy())
    np.testing.assert_array_equal(got.T, ref_codes[:p])
    if to == O.E4M3:
        np.testing.assert_array_equal(sc.cpu().numpy(), ref_scale)


@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
def test_column_norms_quantized(gpu, to):
    A32, Adeq, Ad, sc = quantized_problem(517, 3001, 1, 5, to)
    got = gpu.column_norms(Ad, col_scale=sc).cpu().numpy()
    np.testing.assert_allclose(got, np.sqrt((Adeq ** 2).sum(axis=0)), rtol=1e-12)


# (form, m, p, n, seed): one, two and four component blocks; ragged p (not a
# multiple of the 8/16-row slot) and n (not a multiple of the 64-column chunk)
CASES = [
    (O.SL1, 1, 1003, 5011, 1),
    (O.SL0, 1, 2047, 3001, 2),
    (O.BL1, 8, 1000, 4099, 3),
    (O.BL0, 5, 1537, 2000, 4),
    (O.BL1, 20, 301, 1500, 5),
    (O.BL0, 40, 260, 1200, 6),
    (O.BL1, 3, 13, 700, 7),
]


def _cid(c):
    return f"{FORM_NAMES[c[0]]}-m{c[1]}-p{c[2]}-n{c[3]}"


# correlation kernel variants: one wave per workgroup (q), and four waves
# sharing each X stage (qw: the default 2 stages of 8-tile chunks, 3 stages of
# 4-tile chunks, 2 stages of 4-tile chunks)
QVARIANTS = ["q", "qw", "qw-3", "qw-2"]


def _set_variant(kernel, monkeypatch):
    if kernel == "q":
        monkeypatch.setenv("GPSPCA_CORR_KERNEL", "mfma")
    else:
        monkeypatch.setenv("GPSPCA_CORR_KERNEL", "qw")
    if "-" in kernel:
        monkeypatch.setenv("GPSPCA_MFMA_STAGES", kernel.split("-")[1])


@pytest.mark.parametrize("kernel", QVARIANTS)
@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
@pytest.mark.parametrize("case", CASES, ids=_cid)
def test_step_parity_quantized(gpu, case, to, kernel, monkeypatch):
    """One pass on the codes against the oracle on the dequantized matrix, for
    every variant of the correlation kernel."""
    form, m, p, n, seed = case
    _set_variant(kernel, monkeypatch)
    print(f"\n[quant step] {kernel} {TNAME[to]} {_cid(case)}", flush=True)
    A32, Adeq, Ad, sc = quantized_problem(p, n, m, seed, to)
    mu = np.linspace(1.0, 0.7, m) if form >= O.BL1 else None
    X0 = fp32_round(O.init(Adeq, m)[0])
    g0 = W.gamma_absolute(Adeq, is_l0(form), 0.02 if is_l0(form) else 0.05)
    gamma = pick_gamma(Adeq, form, m, mu, X0, g0, iters=1)
    ref = O.step(Adeq, form, X0, gamma, mu=mu)
    out = gpu.step(Ad, form, x_to_device(X0), gamma, mu=None if mu is None else list(mu),
                   col_scale=sc)
    S = out.S.cpu().numpy().astype(np.float64)
    ties = tie_mask(Adeq, X0, form, gamma, mu)
    if is_l0(form):
        assert not ties.any()
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    eb = corr_band(Adeq, X0) * (np.ones(m) if mu is None else mu)[None, :]
    assert np.all(np.abs(S - ref["S"]) <= 2 * eb + 1e-7 * np.abs(ref["S"]))
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5, atol=1e-9 * max(1.0, ref["F"]))


@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
@pytest.mark.parametrize("form,m", [(O.SL1, 1), (O.SL0, 1), (O.BL1, 8), (O.BL0, 4)])
def test_solve_parity_quantized(gpu, form, m, to):
    p, n, iters = 900, 3000, 10
    print(f"\n[quant solve] {TNAME[to]} {FORM_NAMES[form]} m={m}", flush=True)
    A32, Adeq, Ad, sc = quantized_problem(p, n, m, 11 + m, to)
    X0 = fp32_round(O.init(Adeq, m)[0])
    g0 = W.gamma_absolute(Adeq, is_l0(form), 0.03 if is_l0(form) else 0.06)
    gamma = pick_gamma(Adeq, form, m, None, X0, g0, iters=iters)
    ref = O.solve(Adeq, form, m, gamma, X0=X0, tol=0.0, max_iter=iters)
    res = gpu.solve(Ad, form, m, gamma, X0=x_to_device(X0), tol=0.0, max_iter=iters,
                    col_scale=sc)
    assert res.n_iter == ref["n_iter"] and res.status == ref["status"]
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=1e-5)
    assert rel(res.X.cpu().numpy(), ref["X"]) <= 1e-5
    Z = res.Z.cpu().numpy().astype(np.float64)
    for j in range(m):
        assert rel(Z[:, j], ref["Z"][:, j]) <= 1e-5
    ties = tie_mask(Adeq, ref["X"], form, gamma, None)
    np.testing.assert_array_equal(res.support_mask().cpu().numpy()[~ties], ref["support"][~ties])


@pytest.mark.parametrize("kernel", ["q", "qw"])
@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
def test_path_quantized_columns_match_oracle(gpu, to, kernel, monkeypatch):
    _set_variant(kernel, monkeypatch)
    p, n, K, iters = 700, 4000, 32, 8
    A32, Adeq, Ad, sc = quantized_problem(p, n, 1, 21, to)
    fr = W.gamma_fractions(K)
    cmax = float(np.sqrt((Adeq ** 2).sum(axis=0)).max())
    gammas = [float(f * cmax) for f in fr]
    x0 = fp32_round(O.init(Adeq, 1)[0])
    X0 = np.repeat(x0, K, axis=1)
    res = gpu.solve_path(Ad, O.SL1, gammas, X0=x_to_device(X0), tol=0.0, max_iter=iters,
                         col_scale=sc)
    X = res.X.cpu().numpy()
    for k in (0, 9, 20, 31):
        ref = O.solve(Adeq, O.SL1, 1, gammas[k], X0=x0, tol=0.0, max_iter=iters)
        assert res.n_iter[k] == ref["n_iter"]
        np.testing.assert_allclose(res.traces[k], ref["trace"], rtol=1e-5)
        assert rel(X[:, k], ref["X"][:, 0]) <= 1e-5


@pytest.mark.parametrize("form,m", [(O.SL1, 1), (O.SL0, 1), (O.BL1, 6), (O.BL0, 3)])
def test_refine_from_oracle_inputs(gpu, form, m):
    """Frozen-support FP32 passes from the oracle's bf16 result."""
    p, n, passes = 800, 3500, 5
    A32, Adeq, _, _ = quantized_problem(p, n, m, 31 + m, O.BF16)
    A64 = A32.astype(np.float64)
    X0 = fp32_round(O.init(Adeq, m)[0])
    g0 = W.gamma_absolute(Adeq, is_l0(form), 0.03 if is_l0(form) else 0.06)
    gamma = pick_gamma(Adeq, form, m, None, X0, g0, iters=12)
    q = O.solve(Adeq, form, m, gamma, X0=X0, tol=0.0, max_iter=12)
    Xq = fp32_round(q["X"])
    sup = q["support"].reshape(n, m)
    gamma_r = gamma
    ref = O.solve(A64, form, m, gamma_r, X0=Xq, tol=0.0, max_iter=passes, mask=sup)
    res = gpu.refine(to_device(A32), form, m, gamma_r, _words_to_device(sup), x_to_device(Xq),
                     tol=0.0, max_iter=passes)
    assert res.n_iter == ref["n_iter"]
    np.testing.assert_allclose(res.trace, ref["trace"], rtol=1e-5)
    assert rel(res.X.cpu().numpy(), ref["X"]) <= 1e-5
    got = res.support_mask().cpu().numpy()
    assert not np.any(got & ~sup)
    ties = tie_mask(A64, ref["X"], form, gamma_r, None)
    np.testing.assert_array_equal(got[~ties], ref["support"][~ties])


def test_refine_path_from_oracle_inputs(gpu):
    p, n, K, passes = 600, 3000, 6, 5
    A32, Adeq, _, _ = quantized_problem(p, n, 1, 41, O.E4M3)
    A64 = A32.astype(np.float64)
    cmax = float(np.sqrt((Adeq ** 2).sum(axis=0)).max())
    gammas = [float(f * cmax) for f in W.gamma_fractions(K, 0.03, 0.3)]
    x0 = fp32_round(O.init(Adeq, 1)[0])
    Xs, sups, refs = [], [], []
    for g in gammas:
        q = O.solve(Adeq, O.SL1, 1, g, X0=x0, tol=0.0, max_iter=10)
        Xs.append(fp32_round(q["X"]))
        sups.append(q["support"].reshape(n, 1))
        refs.append(O.solve(A64, O.SL1, 1, g, X0=Xs[-1], tol=0.0, max_iter=passes, mask=sups[-1]))
    sup = np.concatenate(sups, axis=1)
    res = gpu.refine_path(to_device(A32), O.SL1, gammas, _words_to_device(sup),
                          x_to_device(np.concatenate(Xs, axis=1)), tol=0.0, max_iter=passes)
    X = res.X.cpu().numpy()
    for k in range(K):
        assert res.n_iter[k] == refs[k]["n_iter"]
        np.testing.assert_allclose(res.traces[k], refs[k]["trace"], rtol=1e-5)
        assert rel(X[:, k], refs[k]["X"][:, 0]) <= 1e-5


@pytest.mark.parametrize("to", [O.BF16, O.E4M3], ids=["bf16", "e4m3"])
def test_quantized_solve_then_refine_accuracy(gpu, to):
    """End to end on the GPU: quantize, solve to tol 1e-6, 5 FP32 passes on the
    found support.  The error against the FP64 oracle on the original A is
    printed for SL1 and SL0 over 4 gammas each (a planted spike, beta =
    10 sqrt(pn), k = 50).  How close 5 passes get depends on the restricted spectral gap, so
    the assertion is a loose bound; the printed figures are the measurement."""
    p, n, refine = 1000, 10000, 5
    A32, _, _, _ = W.planted_single(p, n, 57, k=50, beta=10.0 * np.sqrt(p * n))
    A64 = A32.astype(np.float64)
    Ad = to_device(A32)
    Aq, sc = gpu.quantize(Ad, TD[to])
    cmax = float(np.sqrt((A64 ** 2).sum(axis=0)).max())
    worst = dict(x_q=0.0, x=0.0, z=0.0, F=0.0, sup=0)
    # fractions that keep the supports on the planted columns (away from the
    # noise correlations, whose thresholds quantization may move)
    for form, lo, hi in ((O.SL1, 0.15, 0.45), (O.SL0, 0.02, 0.2)):
        for f in W.gamma_fractions(4, lo, hi):
            g = float(f * (cmax * cmax if is_l0(form) else cmax))
            ref = O.solve(A64, form, 1, g, tol=1e-6, max_iter=1000)
            q = gpu.solve(Aq, form, 1, g, tol=1e-6, max_iter=1000, col_scale=sc)
            r = gpu.refine(Ad, form, 1, g, q.support, q.X, tol=0.0, max_iter=refine)
            x = r.X.cpu().numpy()[:, 0].astype(np.float64)
            sgn = 1.0 if x @ ref["X"][:, 0] >= 0 else -1.0
            worst["x_q"] = max(worst["x_q"], rel(sgn * q.X.cpu().numpy()[:, 0], ref["X"][:, 0]))
            worst["x"] = max(worst["x"], rel(sgn * x, ref["X"][:, 0]))
            worst["z"] = max(worst["z"], rel(sgn * r.Z.cpu().numpy()[:, 0], ref["Z"][:, 0]))
            worst["F"] = max(worst["F"], abs(r.trace[-1] - ref["trace"][-1]) / ref["trace"][-1])
            worst["sup"] = max(worst["sup"], int((r.support_mask().cpu().numpy()[:, 0]
                                                  != ref["support"][:, 0]).sum()))
    print(f"\n[accuracy] {TNAME[to]} vs FP64 oracle on the FP32 matrix (worst of 8 solves): "
          f"x {worst['x_q']:.2e} before / {worst['x']:.2e} after {refine} refinement passes, "
          f"z {worst['z']:.2e}, F {worst['F']:.2e}, support differences {worst['sup']}",
          flush=True)
    assert worst["sup"] == 0
    assert worst["x"] <= worst["x_q"] + 1e-6
    assert worst["x"] <= 1e-4 and worst["F"] <= 1e-4
