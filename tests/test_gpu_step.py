"""Step parity: one pass of the HIP path (gpspca_step through the C ABI) against
the FP64 oracle at the same FP32 point X, element by element.

Supports must match exactly (gamma is placed so that no margin lies within
8x the FP32 forward-error band of the correlation); thresholded values within
the band; G and the objective within 1e-5 relative."""
import numpy as np
import pytest

import oracle as O
from workloads import generators as W

from _util import (FORM_NAMES, corr_band, fp32_round, is_l0, pick_gamma, rel, tie_mask,
                   to_device, x_to_device)

pytestmark = pytest.mark.gpu

# (form, m, p, n, lda_extra, seed): covers the fused m = 1 kernel (several
# thread counts, ragged row quads), the block path with 1, 2 and 3 component
# groups, the non-vector path (lda not a multiple of 4) and p > 20480 (m = 1 on
# the block kernels).
CASES = [
    (O.SL1, 1, 1003, 5011, 0, 1),
    (O.SL0, 1, 1003, 5011, 0, 2),
    (O.SL1, 1, 4999, 3001, 0, 3),
    (O.SL0, 1, 4999, 3001, 1, 4),
    (O.SL1, 1, 90, 2000, 0, 5),
    (O.SL0, 1, 21003, 700, 0, 6),
    (O.BL1, 1, 777, 1500, 0, 7),
    (O.BL1, 3, 517, 4099, 0, 8),
    (O.BL0, 3, 517, 4099, 3, 9),
    (O.BL1, 8, 2050, 3333, 0, 10),
    (O.BL0, 8, 2050, 3333, 0, 11),
    (O.BL1, 13, 301, 2000, 0, 12),
    (O.BL0, 20, 300, 1500, 2, 13),
    (O.BL1, 64, 200, 900, 0, 14),
    # matrix-core correlation path (lda % 4 == 0): ragged tails, 1/2/4
    # component blocks of 16, m = 1 with p > 20480, n smaller than one tile
    (O.BL1, 8, 2051, 3333, 1, 15),
    (O.BL0, 8, 2048, 3000, 0, 16),
    (O.BL0, 20, 300, 1500, 0, 17),
    (O.BL1, 33, 257, 1000, 3, 18),
    (O.SL1, 1, 20996, 600, 0, 19),
    (O.BL0, 5, 1002, 37, 2, 20),
    (O.BL1, 2, 3, 500, 1, 21),
    (O.BL0, 6, 12004, 400, 0, 22),   # m <= 8 with p > 10240: matrix-core path
]


def _ids(c):
    return f"{FORM_NAMES[c[0]]}-m{c[1]}-p{c[2]}-n{c[3]}-ldx{c[4]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_step_parity(gpu, case):
    form, m, p, n, extra, seed = case
    print(f"\n[step] {_ids(case)} seed={seed}", flush=True)
    A32, _, _ = W.planted_block(p, n, min(m, 4), seed, k=min(50, n // 8))
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.6, m) if form >= O.BL1 else np.ones(1)
    X0 = fp32_round(O.init(A64, m)[0])
    frac = 0.05 if not is_l0(form) else 0.02
    g0 = W.gamma_absolute(A64, is_l0(form), frac)
    gamma = pick_gamma(A64, form, m, mu, X0, g0, iters=1)
    ref = O.step(A64, form, X0, gamma, mu=mu if form >= O.BL1 else None)

    Ad = to_device(A32, lda=p + extra)
    out = gpu.step(Ad, form, x_to_device(X0), gamma, mu=list(mu) if form >= O.BL1 else None)
    S = out.S.cpu().numpy().astype(np.float64)
    G = out.G.cpu().numpy()

    ties = tie_mask(A64, X0, form, gamma, mu if form >= O.BL1 else None)
    if is_l0(form):
        assert not ties.any()
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    nt = ties.sum(axis=0)
    assert np.all(np.abs(np.asarray(out.nnz) - ref["nnz"]) <= nt)
    eb = corr_band(A64, X0)
    sb = eb * mu[None, :] + 1e-7 * np.abs(ref["S"])
    assert np.all(np.abs(S - ref["S"]) <= sb)
    assert rel(G, ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5, atol=1e-9 * max(1.0, ref["F"]))


@pytest.mark.parametrize("form", [O.SL1, O.SL0, O.BL1, O.BL0])
def test_step_zero_gamma_dense_support(gpu, form):
    """gamma = 0: every entry is active, the back-projection is a full GEMM."""
    p, n = 333, 2500
    m = 1 if form < O.BL1 else 5
    A32 = W.gaussian(p, n, 21)
    A64 = A32.astype(np.float64)
    X0 = fp32_round(W.random_orthonormal(p, m, 22))
    mu = np.ones(m)
    ref = O.step(A64, form, X0, 0.0, mu=mu if form >= O.BL1 else None)
    out = gpu.step(to_device(A32), form, x_to_device(X0), 0.0)
    assert list(out.nnz) == [n] * m
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)


@pytest.mark.parametrize("kernel", ["vx", "mv", "mfma", "mfma-fullx", "rd", "rd128", "wg", "x3",
                                    "valu"])
@pytest.mark.parametrize("form,m", [(O.BL1, 4), (O.BL0, 8)])
def test_every_correlation_kernel(gpu, kernel, form, m, monkeypatch):
    """Force each block correlation kernel (registers-X, matrix cores through
    registers, matrix cores through LDS DMA, FP32 split into bfloat16 parts on
    the bfloat16 matrix cores, plain vector ALU) on the same case: one step and
    a 6-pass solve against the oracle."""
    monkeypatch.setenv("GPSPCA_CORR_KERNEL", kernel.split("-")[0])
    if kernel == "mfma-fullx":
        # X staged for all 16 component slots (m <= 8 stages 8 of them by default)
        monkeypatch.setenv("GPSPCA_MFMA_HALF_X", "0")
    p, n = 1003, 3001  # ragged row quad
    A32, _, _ = W.planted_block(p, n, 3, 23, k=40)
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.7, m)
    X0 = fp32_round(O.init(A64, m)[0])
    g0 = W.gamma_absolute(A64, is_l0(form), 0.02 if is_l0(form) else 0.05)
    gamma = pick_gamma(A64, form, m, mu, X0, g0, iters=6)
    Ad = to_device(A32, lda=p + 1)  # lda % 4 == 0: every kernel is eligible
    ref = O.step(A64, form, X0, gamma, mu=mu)
    out = gpu.step(Ad, form, x_to_device(X0), gamma, mu=list(mu))
    ties = tie_mask(A64, X0, form, gamma, mu)
    S = out.S.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)
    rs = O.solve(A64, form, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=6)
    res = gpu.solve(Ad, form, m, gamma, mu=list(mu), X0=x_to_device(X0), tol=0.0, max_iter=6)
    assert rel(res.X.cpu().numpy(), rs["X"]) <= 1e-5
    np.testing.assert_allclose(res.trace, rs["trace"], rtol=1e-5)


@pytest.mark.parametrize("kernel", ["rd", "rd128", "x3", "x3-d3"])
@pytest.mark.parametrize("m,p,n", [(20, 1001, 2999), (40, 514, 1500), (16, 4097, 64),
                                   (64, 2003, 1203)])
def test_register_direct_kernels_component_groups(gpu, kernel, m, p, n, monkeypatch):
    """The register-direct matrix-core kernels (FP32, and FP32 split into
    bfloat16 parts with 2 or 3 stages in flight) with 1, 2 and 4 component
    groups, ragged rows and a matrix of only 4 tiles: one step against the
    oracle."""
    monkeypatch.setenv("GPSPCA_CORR_KERNEL", kernel.split("-")[0])
    if kernel.endswith("-d3"):
        monkeypatch.setenv("GPSPCA_MFMA_STAGES", "3")
    print(f"\n[corr {kernel}] m={m} p={p} n={n}", flush=True)
    A32, _, _ = W.planted_block(p, n, 4, 90 + m, k=min(40, n // 4))
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.7, m)
    X0 = fp32_round(O.init(A64, m)[0])
    gamma = W.gamma_absolute(A64, False, 0.05)
    Ad = to_device(A32, lda=(p + 3) // 4 * 4)
    ref = O.step(A64, O.BL1, X0, gamma, mu=mu)
    out = gpu.step(Ad, O.BL1, x_to_device(X0), gamma, mu=list(mu))
    ties = tie_mask(A64, X0, O.BL1, gamma, mu)
    S = out.S.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    # thresholded values within the FP32 band of the correlation
    eb = corr_band(A64, X0) * mu[None, :]
    assert np.all(np.abs(S - ref["S"]) <= eb + 1e-7 * np.abs(ref["S"]))
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)


@pytest.mark.parametrize("stages", ["3", "8"])
@pytest.mark.parametrize("m,p,n", [(20, 1003, 3001), (32, 2050, 1999), (17, 257, 700)])
def test_matrix_core_two_groups_stage_variants(gpu, stages, m, p, n, monkeypatch):
    """The LDS-DMA matrix-core kernel with two component groups, in chunks of
    up to 4 tiles (3 stages) and of up to 8 tiles (2 stages): one step against
    the oracle, with ragged rows and ragged tiles."""
    monkeypatch.setenv("GPSPCA_CORR_KERNEL", "mfma")
    monkeypatch.setenv("GPSPCA_MFMA_STAGES", stages)
    print(f"\n[corr mfma stages={stages}] m={m} p={p} n={n}", flush=True)
    A32, _, _ = W.planted_block(p, n, 4, 120 + m, k=min(40, n // 4))
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.7, m)
    X0 = fp32_round(O.init(A64, m)[0])
    gamma = W.gamma_absolute(A64, False, 0.05)
    Ad = to_device(A32, lda=(p + 3) // 4 * 4)
    ref = O.step(A64, O.BL1, X0, gamma, mu=mu)
    out = gpu.step(Ad, O.BL1, x_to_device(X0), gamma, mu=list(mu))
    ties = tie_mask(A64, X0, O.BL1, gamma, mu)
    S = out.S.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)


# (form, m, p, n, waves per CU, lda extra): more tiles of 16 columns than
# waves, so the matrix-core correlation takes q whole tiles per wave and splits
# the leftover tiles by rows over all waves.  Covers q = 1, 2 and 7, components
# in one half stage (m <= 8) and a full group (m = 16), ragged row quads, a
# ragged last tile among the leftover ones, matrices of 2 row stages, and two
# component groups (m = 20, 32).
BAL_CASES = [
    (O.BL1, 8, 300, 20000, 4, 0),
    (O.BL0, 5, 301, 20000, 4, 3),
    (O.BL1, 8, 67, 5000, 1, 1),
    (O.BL1, 16, 1000, 9000, 2, 0),
    (O.BL0, 3, 2000, 40003, 4, 0),
    (O.BL1, 8, 129, 30277, 1, 3),
    (O.BL1, 20, 300, 20000, 4, 0),
    (O.BL0, 32, 257, 9000, 2, 3),
]


@pytest.mark.parametrize("balance", ["1", "0"])
@pytest.mark.parametrize("case", BAL_CASES, ids=lambda c: f"{FORM_NAMES[c[0]]}-m{c[1]}-p{c[2]}-n{c[3]}-w{c[4]}")
def test_matrix_core_balanced_partition(gpu, case, balance, monkeypatch):
    """Leftover tiles split by rows over the waves (and, for comparison, the
    partition in whole tiles only): one step and a 4-pass solve against the
    oracle."""
    import torch
    form, m, p, n, wpc, extra = case
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    ntile = (n + 15) // 16
    q, rem = divmod(ntile, ncu * wpc)
    assert q >= 1 and rem > 0 and q + 1 <= 8   # the case exercises the split
    monkeypatch.setenv("GPSPCA_CORR_KERNEL", "mfma")
    monkeypatch.setenv("GPSPCA_MFMA_WAVES_PER_CU", str(wpc))
    monkeypatch.setenv("GPSPCA_MFMA_BALANCE", balance)
    print(f"\n[corr balanced={balance}] m={m} p={p} n={n} waves={ncu * wpc} q={q} rem={rem}",
          flush=True)
    A32, _, _ = W.planted_block(p, n, min(m, 4), 140 + m, k=40)
    A64 = A32.astype(np.float64)
    mu = np.linspace(1.0, 0.7, m)
    X0 = fp32_round(O.init(A64, m)[0])
    g0 = W.gamma_absolute(A64, is_l0(form), 0.02 if is_l0(form) else 0.05)
    gamma = pick_gamma(A64, form, m, mu, X0, g0, iters=4)
    Ad = to_device(A32, lda=(p + extra + 3) // 4 * 4)
    ref = O.step(A64, form, X0, gamma, mu=mu)
    out = gpu.step(Ad, form, x_to_device(X0), gamma, mu=list(mu))
    ties = tie_mask(A64, X0, form, gamma, mu)
    S = out.S.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal((S != 0)[~ties], (ref["S"] != 0)[~ties])
    eb = corr_band(A64, X0) * mu[None, :]
    assert np.all(np.abs(S - ref["S"]) <= eb + 1e-7 * np.abs(ref["S"]))
    assert rel(out.G.cpu().numpy(), ref["G"]) <= 1e-5
    np.testing.assert_allclose(out.f, ref["f"], rtol=1e-5)
    assert list(out.nnz) == list(ref["nnz"]) or ties.any()
    rs = O.solve(A64, form, m, gamma, mu=mu, X0=X0, tol=0.0, max_iter=4)
    res = gpu.solve(Ad, form, m, gamma, mu=list(mu), X0=x_to_device(X0), tol=0.0, max_iter=4)
    assert rel(res.X.cpu().numpy(), rs["X"]) <= 1e-5
    np.testing.assert_allclose(res.trace, rs["trace"], rtol=1e-5)
