"""gpspca_solve_noalloc (the solve with the library's own device scratch) against
gpspca_solve (caller workspace) through the C ABI: the same kernels run in the
same order, so X, Z, the support words, the trace, the pass count and the
status must be bitwise equal.  Two calls in a row on one GPU, the second on a
smaller problem (the scratch keeps the first call's contents, so everything the
second reads must be initialized by the call itself), then a problem too large
for the scratch, which must be rejected before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from workloads import generators as W

from _util import to_device

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.n_iter == b.n_iter and a.status == b.status
    assert a.trace == b.trace
    assert bool((a.X == b.X).all()) and bool((a.Z == b.Z).all())
    assert bool((a.support == b.support).all())


@pytest.mark.parametrize("first,second", [
    ((O.BL1, 8, 1500, 6000, 0.04), (O.SL0, 1, 700, 2000, 0.02)),
    ((O.BL0, 16, 900, 5000, 0.01), (O.BL1, 4, 300, 1200, 0.05)),
])
def test_noalloc_matches_workspace_solve(gpu, first, second):
    for form, m, p, n, frac in (first, second):
        print(f"\n[noalloc] form={form} m={m} p={p} n={n}", flush=True)
        A32, _, _ = W.planted_block(p, n, min(m, 4), 5 + m, k=40)
        Ad = to_device(A32)
        g = W.gamma_absolute(A32.astype(np.float64), form in (O.SL0, O.BL0), frac)
        mu = list(np.linspace(1.0, 0.7, m)) if form >= O.BL1 else None
        ref = gpu.solve(Ad, form, m, g, mu=mu, tol=1e-5, max_iter=40)
        got = gpu.solve_noalloc(Ad, form, m, g, mu=mu, tol=1e-5, max_iter=40)
        _same(got, ref)
        # fixed passes from an explicit start
        ref = gpu.solve(Ad, form, m, g, mu=mu, X0=ref.X.contiguous(), tol=0.0, max_iter=9)
        got = gpu.solve_noalloc(Ad, form, m, g, mu=mu, X0=got.X.contiguous(), tol=0.0,
                                max_iter=9)
        _same(got, ref)


def test_noalloc_rejects_problems_larger_than_its_scratch(gpu):
    """n x m FP32 thresholded values alone exceed the scratch here."""
    import paper_1312_6182_amd as G
    p, n, m = 64, 300000, 64
    assert 4 * n * m > G.NOALLOC_SCRATCH_BYTES
    Ad = torch.zeros((n, p), dtype=torch.float32, device="cuda").t()
    Ad[0, :] = 1.0
    with pytest.raises(G.GpspcaError) as e:
        gpu.solve_noalloc(Ad, O.BL1, m, 0.1, tol=0.0, max_iter=2,
                          X0=torch.eye(p, m, device="cuda"))
    assert e.value.code == G.ENOMEM
    assert "GPSPCA_NOALLOC_SCRATCH_BYTES" in G.last_error()
