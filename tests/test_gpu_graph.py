"""Pass pairs replayed from a captured HIP graph give exactly the results of the
same passes enqueued one by one (GPSPCA_GRAPH=0): fixed pass counts and
tolerance-stopped solves (several replays, with the host's polls of the device
stop flag in between), on the fused single-unit pass, the matrix-core block
pass (also with leftover tiles split by rows), a gamma path and bfloat16
storage."""
import numpy as np
import pytest
import torch

from workloads import generators as W

from _util import to_device

pytestmark = pytest.mark.gpu


def _run(gpu, monkeypatch, graph, fn):
    monkeypatch.setenv("GPSPCA_GRAPH", "1" if graph else "0")
    return fn()


@pytest.mark.parametrize("case", ["m1", "block", "block-bal", "path", "bf16"])
@pytest.mark.parametrize("tol,iters", [(0.0, 21), (1e-6, 400)])
def test_graph_replay_equals_eager(gpu, monkeypatch, case, tol, iters):
    if case == "block-bal":
        # more tiles of 16 columns than correlation waves: the leftover tiles
        # are split by rows and finished by a second kernel in every pass
        A32, _, _ = W.planted_block(300, 20000, 4, 78, k=40)
    else:
        A32, _, _ = W.planted_block(900, 7000, 4, 77, k=40)
    Ad = to_device(A32)
    g = W.gamma_absolute(A32.astype(np.float64), False, 0.05)
    if case == "m1":
        fn = lambda: gpu.solve(Ad, 0, 1, g, tol=tol, max_iter=iters)
    elif case in ("block", "block-bal"):
        fn = lambda: gpu.solve(Ad, 2, 8, g, tol=tol, max_iter=iters)
    elif case == "path":
        gs = [g * f for f in (0.5, 1.0, 1.5, 2.0, 3.0)]
        fn = lambda: gpu.solve_path(Ad, 0, gs, tol=tol, max_iter=iters)
    else:
        Aq, _ = gpu.quantize(Ad, torch.bfloat16)
        fn = lambda: gpu.solve(Aq, 2, 4, g, tol=tol, max_iter=iters)
    eager = _run(gpu, monkeypatch, False, fn)
    for _ in range(2):   # two graph solves, each replaying the captured pair many times
        rep = _run(gpu, monkeypatch, True, fn)
        np.testing.assert_array_equal(rep.X.cpu().numpy(), eager.X.cpu().numpy())
        np.testing.assert_array_equal(rep.Z.cpu().numpy(), eager.Z.cpu().numpy())
        if case == "path":
            assert rep.n_iter == eager.n_iter and rep.status == eager.status
            for a, b in zip(rep.traces, eager.traces):
                np.testing.assert_array_equal(np.asarray(a), np.asarray(b))
        else:
            assert rep.n_iter == eager.n_iter and rep.status == eager.status
            np.testing.assert_array_equal(np.asarray(rep.trace), np.asarray(eager.trace))
