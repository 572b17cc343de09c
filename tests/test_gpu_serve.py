"""The solve server on the GPU: mixed requests admitted while others run give
the same results as the same solves run alone through gpspca_solve (bitwise:
every kernel reduces in a fixed order, so concurrency cannot change a
result), match the FP64 oracle, and survive eviction and re-upload."""
import numpy as np
import pytest
import torch

import oracle as O
from workloads import generators as W

from _util import fp32_round, is_l0, pick_gamma_starts, rel, to_device

pytestmark = pytest.mark.gpu


def _alone(gpu, A32, store, form, m, gamma, mu, tol, max_iter):
    Ad = to_device(A32)
    if store == "bf16":
        Ad, _ = gpu.quantize(Ad, torch.bfloat16)
    if form < 2 and m > 1:
        return gpu.solve_multistart(Ad, form, m, gamma, tol=tol, max_iter=max_iter)
    return gpu.solve(Ad, form, m, gamma, mu=mu, tol=tol, max_iter=max_iter)


def _same_as_solo(r, solo):
    """A served result equals the library's own solve of the same request bitwise."""
    if isinstance(solo.n_iter, list):      # multi-start
        assert r.col_n_iter == solo.n_iter and r.col_status == solo.status
        assert r.n_iter == max(solo.n_iter)
        for a, b in zip(r.trace, solo.traces):
            np.testing.assert_array_equal(np.asarray(a), np.asarray(b))
    else:
        assert r.status == solo.status and r.n_iter == solo.n_iter
        np.testing.assert_array_equal(np.asarray(r.trace), np.asarray(solo.trace))
    np.testing.assert_array_equal(r.X, solo.X.cpu().numpy())
    np.testing.assert_array_equal(r.Z, solo.Z.cpu().numpy())
    np.testing.assert_array_equal(r.support.view(np.int32), solo.support.cpu().numpy())


def _mix(seed):
    rng = np.random.default_rng(seed)
    shapes = [(300, 4000, "f32"), (1500, 2500, "bf16"), (64, 9000, "f32"), (777, 3001, "bf16")]
    mats = [W.planted_single(p, n, seed + i, k=max(10, n // 100), beta=5 * np.sqrt(n))[0]
            for i, (p, n, _) in enumerate(shapes)]
    reqs = []
    for r in range(14):
        i = int(rng.integers(len(mats)))
        form = int(rng.integers(4))
        m = int(rng.choice([1, 4, 16]))        # single-unit forms: m starts
        frac = float(rng.uniform(0.01, 0.5)) if form in (0, 2) else float(rng.uniform(0.005, 0.1))
        A64 = mats[i].astype(np.float64)
        gamma = W.gamma_absolute(A64, is_l0(form), frac)
        mu = list(np.linspace(1.0, 0.5, m)) if form >= 2 and r % 2 else None
        reqs.append((i, form, m, gamma, mu))
    return shapes, mats, reqs


def test_mixed_requests_equal_solo_solves(gpu):
    from paper_1312_6182_amd.serve import Server
    shapes, mats, reqs = _mix(100)
    with Server(2 << 30, slots=4) as srv:
        ids = [srv.register(A, store=s[2]) for A, s in zip(mats, shapes)]
        rids = [srv.submit(ids[i], form, m, g, mu=mu, tol=1e-4, max_iter=200)
                for (i, form, m, g, mu) in reqs]
        res = [srv.wait(r) for r in rids]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["uploads"] == len(mats)
    overlapped = sum(1 for a in res for b in res
                     if a is not b and a.t_admit < b.t_done and b.t_admit < a.t_done)
    print(f"\n[serve] {len(reqs)} requests, {overlapped} overlapping pairs, stats {st}", flush=True)
    # continuous batching: requests admitted while others were on the device
    assert overlapped > 0
    assert sum(1 for r in res[1:] if r.t_admit > min(x.t_admit for x in res)
               and any(o.t_admit < r.t_admit < o.t_done for o in res if o is not r)) > 0
    assert any(form < 2 and m > 1 for (_, form, m, _, _) in reqs)
    for (i, form, m, g, mu), r in zip(reqs, res):
        solo = _alone(gpu, mats[i], shapes[i][2], form, m, g, mu, 1e-4, 200)
        _same_as_solo(r, solo)


def test_served_results_match_the_oracle(gpu):
    from paper_1312_6182_amd.serve import Server
    A32, _, _, _ = W.planted_single(400, 3000, 7, k=30, beta=10 * np.sqrt(400 * 3000))
    A64 = A32.astype(np.float64)
    with Server(1 << 30, slots=2) as srv:
        mid = srv.register(A32)
        cases = [(O.SL1, 1, 0.2), (O.SL0, 1, 0.05), (O.BL1, 3, 0.1), (O.BL0, 2, 0.02)]
        rids = []
        for form, m, frac in cases:
            g = W.gamma_absolute(A64, is_l0(form), frac)
            rids.append((srv.submit(mid, form, m, g, tol=0.0, max_iter=15), form, m, g))
        for rid, form, m, g in rids:
            r = srv.wait(rid)
            ref = O.solve(A64, form, m, g, X0=fp32_round(O.init(A64, m)[0]), tol=0.0, max_iter=15)
            assert r.n_iter == ref["n_iter"]
            np.testing.assert_allclose(r.trace, ref["trace"], rtol=1e-5)
            assert rel(r.X, ref["X"]) <= 1e-5
            np.testing.assert_array_equal(r.support_mask(), ref["support"])


def test_eviction_and_reupload(gpu):
    """An arena that holds about two of the matrices: later requests evict idle
    ones and re-upload them, with unchanged results."""
    from paper_1312_6182_amd.serve import Server
    mats = [W.gaussian(1000, 20000, 60 + i) for i in range(3)]   # 80 MB each
    mb = 1 << 20
    with Server(4 * 64 * mb + 180 * mb, slots=4) as srv:   # 180 MB after the staging areas
        ids = [srv.register(A) for A in mats]
        g = [W.gamma_absolute(A.astype(np.float64), False, 0.1) for A in mats]
        order = [0, 1, 2, 0, 1, 2, 0]
        out = []
        for i in order:
            out.append(srv.wait(srv.submit(ids[i], O.SL1, 1, g[i], tol=0.0, max_iter=5)))
        st = srv.stats()
    assert st["evictions"] >= 2 and st["uploads"] > 3
    for k, i in enumerate(order):
        solo = _alone(gpu, mats[i], "f32", O.SL1, 1, g[i], None, 0.0, 5)
        np.testing.assert_array_equal(out[k].X, solo.X.cpu().numpy())


def test_oversized_request_is_rejected(gpu):
    from paper_1312_6182_amd.serve import Server
    import paper_1312_6182_amd as G
    with Server(200 << 20, slots=1) as srv:
        mid = srv.register(W.gaussian(2000, 30000, 3))   # 240 MB > arena
        with pytest.raises(G.GpspcaError) as e:
            srv.submit(mid, O.SL1, 1, 1.0)
        assert e.value.code == G.ENOMEM
        with pytest.raises(G.GpspcaError) as e:
            srv.submit(mid, O.SL1, 65, 1.0)     # more starts than GPSPCA_MAX_M
        assert e.value.code == G.EINVAL


def test_served_multistart_matches_the_oracle(gpu):
    """A single-unit request with m = 4 is 4 starts: start k is the column of
    the k-th largest norm, normalized, and each result is the oracle's
    single-unit solve from it."""
    from paper_1312_6182_amd.serve import Server
    A32, _, _, _ = W.planted_single(500, 4000, 17, k=40, beta=10 * np.sqrt(500 * 4000))
    A64 = A32.astype(np.float64)
    idx = O.top_m(O.column_norms(A64), 4)
    with Server(1 << 30, slots=2) as srv:
        mid = srv.register(A32)
        x0s = [fp32_round(A64[:, [i]] / np.linalg.norm(A64[:, i])) for i in idx]
        for form, frac in ((O.SL1, 0.2), (O.SL0, 0.05)):
            g = pick_gamma_starts(A64, form, x0s, W.gamma_absolute(A64, is_l0(form), frac), 12)
            r = srv.wait(srv.submit(mid, form, 4, g, tol=0.0, max_iter=12))
            for k in range(4):
                ref = O.solve(A64, form, 1, g, X0=x0s[k], tol=0.0, max_iter=12)
                assert r.col_n_iter[k] == ref["n_iter"] and r.col_status[k] == ref["status"]
                np.testing.assert_allclose(r.trace[k], ref["trace"], rtol=1e-5)
                assert rel(r.X[:, k], ref["X"][:, 0]) <= 1e-5
