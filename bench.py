"""Benchmark of the GP-SPCA power iteration on one MI355X.

A step is one full pass of the power iteration (correlation, threshold,
back-projection, fixed-order reductions, FP64 retraction and the on-device
stopping rule) over the block workload A: 10000 x 100000 FP32 (4 GB,
N(0,1) noise plus 8 planted sparse components), m = 8, BL1 with
gamma = 0.05 max ||a_i|| and mu = 1.  A is resident in HBM before timing.

Prints one JSON line with the headline rate (passes/s), the roofline of the
dominant kernel (HBM bytes of A per launch over its HIP-event duration), the
secondary workloads (mu_j = 1/j, m = 64 on a 64-component matrix, single-unit
and deflated forms), the 32-gamma path in FP32 / bfloat16 / e4m3 storage with
its error against the FP64 oracle, the serving mix with a swept arrival rate,
and the FP64 oracle timed on the host's cores on the same A.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GPM iters/s + HBM GB/s at 10k×100k m=8; solves/s, p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
PROFILE_EVERY = 8   # one launch in 8 of the dominant kernel records timing events


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--p", type=int, default=10000)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--m", type=int, default=8)
    ap.add_argument("--form", default="BL1", choices=["SL1", "SL0", "BL1", "BL0"])
    ap.add_argument("--frac", type=float, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary workloads (BL0, m=64, m=1 and the 5000x50000 single-unit case)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-pmax", type=int, default=20000)
    ap.add_argument("--serve-nmax", type=int, default=200000)
    ap.add_argument("--serve-repeat", type=float, default=0.875,
                    help="probability that a request repeats an earlier request's matrix")
    ap.add_argument("--serve-arena-gb", type=float, default=12.0)
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP64-oracle accuracy check of the gamma path")
    ap.add_argument("--c4-only", action="store_true",
                    help="after the headline, run only the 32-gamma path leg (no accuracy check, "
                         "serving or CPU baseline): for profiling its kernels")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default kernel configuration instead of the autotuned one")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline run, the timing sweep of the paper's efficiency "
                         "experiment (Section 4.1, Fig. 3): P = N/10, m = 5, four panels, one JSON line")
    ap.add_argument("--sweep-seeds", type=int, default=20)
    ap.add_argument("--sweep-oracle-seconds", type=float, default=15.0,
                    help="per panel and size, the oracle is timed on instances while its total "
                         "stays under this budget (always at least one instance up to the size "
                         "whose predicted time exceeds it)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run 3 plain device copies (x * 1) of this many MiB; their "
                         "HBM counter readings calibrate FETCH_SIZE / WRITE_SIZE")
    return ap.parse_args()


def column_norm_max(A: np.ndarray) -> float:
    best = 0.0
    step = 8192
    for c in range(0, A.shape[1], step):
        blk = A[:, c:c + step].astype(np.float64)
        best = max(best, float(np.sqrt((blk * blk).sum(axis=0)).max()))
    return best


KERNEL_SOURCE = {"k_corr_mfma": "k_corr_mfma.hip", "k_corr_rd": "k_corr_mfma.hip",
                 "k_corr_x3": "k_corr_mfma.hip", "k_corr_wg": "k_corr_mfma.hip",
                 "k_corr_q": "k_quant.hip", "k_corr_qw": "k_quant.hip",
                 "k_corr": "k_pass.hip", "k_pass_m1": "k_pass.hip"}


def kernel_source_hash(kernel: str) -> str:
    """Hash of the source file that defines `kernel` (traffic counters are only
    reported while they were taken on this exact source)."""
    f = KERNEL_SOURCE.get(kernel, "k_pass.hip")
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_1312_6182_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload_key: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain-copy
    calibration) from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload_key}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        k, sep, v = line.partition(" = ")
        if sep and " " not in k.strip():
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_source_hash(kernel):
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(kernel: str, p: int, n: int, m: int, elem_bytes: int = 4,
                      scaled: bool = False) -> float:
    """HBM bytes one launch of the dominant kernel must move: per column a_i, its
    p entries read (4, 2 or 1 bytes each, plus a 4-byte scale for e4m3) and m FP32
    thresholded values written (plus a 1-byte activity flag for the block
    kernels); X (p x m FP32) read once."""
    per_col = (elem_bytes * p + (4.0 if scaled else 0.0) + 4.0 * m
               + (0.0 if kernel == "k_pass_m1" else 1.0))
    return n * per_col + 4.0 * p * m


def copy_calibration(torch, mib: int):
    """Plain device copies of known size (read 4N bytes, write 4N bytes each),
    for scaling the HBM byte counters."""
    src = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x {mib} MiB read + {mib} MiB written", file=sys.stderr,
          flush=True)


C4_SAMPLE = (0, 8, 16, 24, 31)


def gamma_path_leg(G, torch, W, Ad, A32, cmax, x0, path_passes=10, refine=5, K=32,
                   sample=C4_SAMPLE):
    """32 single-unit problems (gamma fractions log-spaced 0.01 .. 0.5, all from the
    largest-norm column x0) sharing each pass over A, with A stored in FP32,
    bfloat16 and e4m3fn (+ per-column scales), for SL1 and SL0.

    A solve is a fixed number of passes: FP32 storage runs path_passes + refine
    passes; the narrow storage types run path_passes passes on the quantized
    matrix (quantized once, untimed) and then `refine` FP32 passes on the
    support each problem found (gpspca_refine_path on the FP32 matrix).  The
    timed region covers the path and the refinement; solves/s = K / its
    duration.  The sampled columns' X, Z and final objective are kept for the
    accuracy check against the FP64 oracle, which runs after every GPU leg."""
    p, n = Ad.shape
    fr = W.gamma_fractions(K)
    X0 = torch.from_numpy(np.ascontiguousarray(np.repeat(x0.T, K, axis=0).astype(np.float32)))
    X0 = X0.cuda().t()
    res, kept = {}, {}
    for name, dt in (("f32", None), ("bf16", torch.bfloat16), ("e4m3", torch.float8_e4m3fn)):
        if dt is None:
            Aq, sc, es = Ad, None, 4
        else:
            Aq, sc = G.quantize(Ad, dt)
            es = 2 if dt == torch.bfloat16 else 1
        torch.cuda.synchronize()
        for form, fname in ((0, "SL1"), (1, "SL0")):
            gam = [float(f * (cmax * cmax if form == 1 else cmax)) for f in fr]
            first = path_passes + (refine if dt is None else 0)
            w = G.solve_path(Aq, form, gam, X0=X0, tol=0.0, max_iter=2, col_scale=sc)
            if dt is not None:
                G.refine_path(Ad, form, gam, w.support, w.X, tol=0.0, max_iter=refine)
            torch.cuda.synchronize()
            G.profile_read()
            G.profile_enable(True)
            t0 = time.perf_counter()
            r = G.solve_path(Aq, form, gam, X0=X0, tol=0.0, max_iter=first, col_scale=sc)
            G.profile_enable(False)
            rr = None
            if dt is not None:
                rr = G.refine_path(Ad, form, gam, r.support, r.X, tol=0.0, max_iter=refine)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            kms, launches, kname = G.profile_read()
            kb = algorithmic_bytes(kname, p, n, K, es, dt == torch.float8_e4m3fn)
            fin = rr if rr is not None else r
            cols = list(sample)
            kept[(name, form)] = {
                "X": fin.X[:, cols].cpu().numpy().astype(np.float64),
                "Z": fin.Z[:, cols].cpu().numpy().astype(np.float64),
                "F": [fin.traces[k][-1] for k in cols],
                "S": fin.support_mask()[:, cols].cpu().numpy(),
                "Xq": r.X[:, cols].cpu().numpy().astype(np.float64),
                "Zq": r.Z[:, cols].cpu().numpy().astype(np.float64),
                "Fq": [r.traces[k][-1] for k in cols],
                "Sq": r.support_mask()[:, cols].cpu().numpy(),
                "gammas": [gam[k] for k in cols], "fracs": [float(fr[k]) for k in cols]}
            res[f"{name}_{fname}"] = {
                "solves_per_s": K / el, "passes_per_solve": path_passes + refine,
                "solve_iters_per_s": K * (path_passes + refine) / el,
                "kernel": kname, "kernel_us": 1e3 * kms / max(1, launches),
                "kernel_gbps": kb / (kms / max(1, launches) * 1e-3) / 1e9,
                "a_bytes_per_pass": float(p) * n * es}
            print(f"[bench] gamma path {name} {fname}: {res[f'{name}_{fname}']}", file=sys.stderr,
                  flush=True)
            del r, w, rr, fin
        del Aq, sc
        torch.cuda.empty_cache()
    return res, kept


def gamma_path_accuracy(A32, x0, kept, path_passes=10, refine=5, sample=C4_SAMPLE):
    """Errors of the gamma-path results against the FP64 oracle (untimed).

    total: the final result (after refinement for the narrow types) against the
    oracle's path_passes + refine passes on the original matrix from the same
    start; algorithmic (narrow types): the quantized path before refinement
    against the oracle's path_passes passes on the dequantized matrix, whose
    codes the oracle's own quantizer makes.  Per sampled column: relative
    2-norm errors of x and z, relative error of the final objective, and the
    number of columns whose support membership differs from the oracle's."""
    import oracle as O
    A64 = np.asfortranarray(A32, dtype=np.float64)
    p = A32.shape[0]
    refs = {}
    for form in (0, 1):
        g = kept[("f32", form)]["gammas"]
        refs[form] = [O.solve(A64, form, 1, g[i], X0=x0, tol=0.0, max_iter=path_passes + refine)
                      for i in range(len(sample))]
    del A64

    def err(k, X, Z, F, S, rs):
        rows = []
        for i, r in enumerate(rs):
            nz = np.linalg.norm(r["Z"][:, 0])
            Fo = r["trace"][-1]
            rows.append({
                "column": sample[i], "gamma_frac": k["fracs"][i],
                "x": float(np.linalg.norm(X[:, i] - r["X"][:, 0]) / np.linalg.norm(r["X"][:, 0])),
                "z": float(np.linalg.norm(Z[:, i] - r["Z"][:, 0]) / max(nz, 1e-300)),
                "F": float(abs(F[i] - Fo) / max(abs(Fo), 1e-300)),
                "support_diff": int((S[:, i] != r["support"][:, 0]).sum()),
                "support_size": int(r["support"][:, 0].sum())})
        return rows

    out = {}
    for name, to in (("f32", None), ("bf16", O.BF16), ("e4m3", O.E4M3)):
        rec = {}
        for f, fname in ((0, "SL1"), (1, "SL0")):
            k = kept[(name, f)]
            rec[fname] = {"total_vs_fp64_oracle": err(k, k["X"], k["Z"], k["F"], k["S"], refs[f])}
        if to is not None:
            align = 8 if to == O.BF16 else 16
            codes, scale = O.quantize(A32, to, ldq=(p + align - 1) // align * align)
            Adeq = O.dequantize(codes, to, scale, p)
            del codes
            for f, fname in ((0, "SL1"), (1, "SL0")):
                k = kept[(name, f)]
                rs = [O.solve(Adeq, f, 1, k["gammas"][i], X0=x0, tol=0.0, max_iter=path_passes)
                      for i in range(len(sample))]
                rec[fname]["algorithmic_vs_fp64_oracle_on_dequantized"] = err(
                    k, k["Xq"], k["Zq"], k["Fq"], k["Sq"], rs)
            del Adeq
        for fname in ("SL1", "SL0"):
            for key, rows in rec[fname].items():
                worst = {e: max(r[e] for r in rows) for e in ("x", "z", "F")}
                print(f"[bench] gamma path accuracy {name} {fname} {key}: worst {worst}; "
                      f"per column (frac, x, support diff): "
                      f"{[(round(r['gamma_frac'], 4), r['x'], r['support_diff']) for r in rows]}",
                      file=sys.stderr, flush=True)
        out[name] = rec
    return {"sampled_columns": list(sample), "errors": out,
            "protocol": f"{path_passes} path passes (+ {refine} FP32 refinement passes on the "
                        f"found support for bf16/e4m3; FP32 storage runs {path_passes + refine} "
                        f"path passes) vs the FP64 oracle's {path_passes + refine} passes on the "
                        f"original matrix (total) and its {path_passes} passes on the dequantized "
                        f"matrix (algorithmic), same start, tol = 0"}


def serving_leg(W, count, p_max, n_max, repeat, arena_gb, slots=12, seed=1000,
                rates=(0.25, 0.5, 0.75, 1.0, 1.25)):
    """The serving mix through the solve server: every request a default-start
    solve (tol 1e-4, up to 1000 passes) on a planted-spike matrix (k =
    max(10, n/100), beta = 5 sqrt(n)), p log-uniform in [200, p_max], n
    log-uniform in [2000, n_max].  A closed-loop run (all requests at once)
    gives the saturation rate in solves/s; open-loop runs with Poisson arrivals
    at `rates` x that rate give the latency percentiles (finish - arrival,
    including the upload of a matrix that is not resident).  The arena is
    smaller than the distinct matrices together, so admission evicts idle
    matrices (least recently used first).  Each run starts from an empty
    arena."""
    from paper_1312_6182_amd.serve import Server
    reqs = W.serving_requests(count, seed, p_max=p_max, n_max=n_max, repeat=repeat)
    t = time.perf_counter()
    mats = {}
    for r in reqs:
        key = r["matrix_seed"]
        if key not in mats:
            A, _, _, _ = W.planted_single(r["p"], r["n"], key, k=max(10, r["n"] // 100),
                                          beta=5.0 * (r["n"] ** 0.5))
            cmax = float(np.sqrt(np.einsum("ij,ij->j", A, A, dtype=np.float64).max()))
            mats[key] = (A, cmax, r["dtype"])
    gen_s = time.perf_counter() - t
    distinct_gb = sum(A.nbytes / (2 if dt == "bf16" else 1) for A, _, dt in mats.values()) / 1e9
    print(f"[bench] serving mix: {len(mats)} distinct matrices, {distinct_gb:.1f} GB stored, "
          f"generated in {gen_s:.1f} s", file=sys.stderr, flush=True)

    def run(rate):
        rng = np.random.default_rng(seed + 1)
        with Server(int(arena_gb * (1 << 30)), slots=slots) as srv:
            ids = {k: srv.register(A, store=dt) for k, (A, _, dt) in mats.items()}
            t0 = time.perf_counter()
            at = 0.0
            rids = []
            for r in reqs:
                if rate:
                    at += float(rng.exponential(1.0 / rate))
                    delay = t0 + at - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                A, cmax, _ = mats[r["matrix_seed"]]
                g = r["frac"] * (cmax * cmax if r["form"] in (1, 3) else cmax)
                rids.append(srv.submit(ids[r["matrix_seed"]], r["form"], r["m"], g,
                                       tol=1e-4, max_iter=1000))
            res = [srv.wait(x) for x in rids]
            el = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array([x.latency for x in res])
        # peak number of solves on the device at once (admit..done intervals)
        ev = sorted([(x.t_admit, 1) for x in res] + [(x.t_done, -1) for x in res])
        cur = peak = 0
        for _, d in ev:
            cur += d
            peak = max(peak, cur)
        return {"solves_per_s": len(res) / el, "seconds": el,
                "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                "mean_passes": float(np.mean([x.n_iter for x in res])),
                "uploads": st["uploads"], "evictions": st["evictions"],
                "peak_concurrent": peak,
                "status_counts": {str(s): int(c) for s, c in
                                  zip(*np.unique([x.status for x in res], return_counts=True))}}

    closed = run(None)
    print(f"[bench] serving closed loop: {closed}", file=sys.stderr, flush=True)
    sweep = []
    for f in rates:
        rate = f * closed["solves_per_s"]
        o = run(rate)
        o = dict(o, load=f, arrival_rate_per_s=rate)
        sweep.append(o)
        print(f"[bench] serving open loop at {f}x saturation ({rate:.1f}/s): {o}", file=sys.stderr,
              flush=True)
    return {"workload": f"{count} requests, p log-uniform [200, {p_max}], n log-uniform "
                        f"[2000, {n_max}], forms uniform, m in (1, 4, 16) (single-unit forms: m "
                        f"starts), gamma fraction U[0.01, 0.5], FP32 or bf16 storage, each request "
                        f"repeats an earlier matrix with probability {repeat}; {len(mats)} distinct "
                        f"matrices ({distinct_gb:.1f} GB stored), {slots} slots, {arena_gb} GB "
                        f"arena",
            "generation_s": gen_s, "saturation": closed, "open_loop_sweep": sweep}


def time_gpu(G, torch, Ad, form, m, gamma, steps, warmup, mu=None):
    # warm-up run from the default start (top-m norm columns), then the timed
    # run continues from its iterate with exactly `steps` passes (tol = 0).
    w = G.solve(Ad, form, m, gamma, mu=mu, tol=0.0, max_iter=max(1, warmup))
    # the caller's workspace, allocated once (as a serving loop would keep it):
    # a fresh allocation per call measured about 100 us more per solve
    ws = torch.empty(G.workspace_bytes(Ad, form, m, steps) + 256, dtype=torch.uint8,
                     device=Ad.device)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:]
    G.solve(Ad, form, m, gamma, mu=mu, X0=w.X, tol=0.0, max_iter=1, workspace=ws)
    torch.cuda.synchronize()
    G.profile_read()
    # HIP events on the first launch of the dominant kernel and every
    # PROFILE_EVERY-th after it, recorded by the launch itself
    G.profile_enable(True, every=PROFILE_EVERY)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    r = G.solve(Ad, form, m, gamma, mu=mu, X0=w.X, tol=0.0, max_iter=steps, workspace=ws)
    t1.record()
    torch.cuda.synchronize()
    G.profile_enable(False)
    ms = t0.elapsed_time(t1)
    kms, launches, kname = G.profile_read()
    return r, ms, kms, launches, kname


def deflated_leg(G, torch, Ad, gamma, passes, m=5):
    """m single-unit L1 components by deflation, each run for exactly
    `passes` passes (tol = 0): passes per second over the whole call, which
    includes each component's start (deflated column norms, top column) and
    the deflation projection after every pass."""
    G.solve_deflated(Ad, 0, m, gamma, tol=0.0, max_iter=2)
    torch.cuda.synchronize()
    G.profile_read()
    # HIP events on the first launch of the dominant kernel and every
    # PROFILE_EVERY-th after it, recorded by the launch itself
    G.profile_enable(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    r = G.solve_deflated(Ad, 0, m, gamma, tol=0.0, max_iter=passes)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    G.profile_enable(False)
    kms, launches, kname = G.profile_read()
    pp, nn = Ad.shape
    total = sum(r.n_iter)
    return {"components": m, "passes": total, "passes_per_s": total / el,
            "ms_per_component": 1e3 * el / m, "kernel": kname,
            "kernel_gbps": algorithmic_bytes(kname, pp, nn, 1) / (kms / max(1, launches) * 1e-3) / 1e9}


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def oracle_passes(O, A64, form, X, gamma, K, mu=None):
    """K oracle passes (step + retract) from X; returns passes/s."""
    t0 = time.perf_counter()
    done = 0
    for _ in range(K):
        st = O.step(A64, form, X, gamma, mu=mu)
        done += 1
        if st["F"] == 0.0:
            break
        X, _ = O.retract(st["G"], st["nnz"], X)
    return done / (time.perf_counter() - t0)


def cpu_baseline(A32, form_id, m, gamma, K=3, K2=10):
    """The FP64 oracle timed on the host's cores: K passes of the headline
    workload on the whole matrix from the oracle's own default start, once on
    all host threads and once on one; the single-unit 5000 x 50000 workload for
    K2 passes (both thread counts); the 100 x 1000 centred case solved to its
    tolerance.  `value` is the all-thread headline rate."""
    import oracle as O
    from workloads import generators as W
    allt = O.num_threads()
    A64 = np.asfortranarray(A32, dtype=np.float64)
    X, _ = O.init(A64, m)
    v_all = oracle_passes(O, A64, form_id, X, gamma, K)
    print(f"[bench] oracle headline, {allt} threads: {v_all:.3f} passes/s", file=sys.stderr,
          flush=True)
    O.set_threads(1)
    try:
        v_one = oracle_passes(O, A64, form_id, X, gamma, K)
        print(f"[bench] oracle headline, 1 thread: {v_one:.3f} passes/s", file=sys.stderr,
              flush=True)
        del A64
        A2, _, _, _ = W.planted_single(5000, 50000, 0, k=500)
        A2 = np.asfortranarray(A2, dtype=np.float64)
        g2 = 0.05 * float(np.sqrt((A2 * A2).sum(axis=0)).max())
        x2, _ = O.init(A2, 1)
        c2_one = oracle_passes(O, A2, 0, x2, g2, K2)
    finally:
        O.set_threads(allt)
    c2_all = oracle_passes(O, A2, 0, x2, g2, K2)
    del A2
    A1 = W.gaussian_centered(100, 1000, 0)
    g1 = 0.1 * float(np.sqrt((A1 * A1).sum(axis=0)).max())
    t0 = time.perf_counter()
    r1 = O.solve(A1, 0, 1, g1, tol=1e-4, max_iter=1000)
    c1_s = time.perf_counter() - t0
    return {
        "value": v_all,
        "unit": "iters/s",
        "cores": allt,
        "kind": "oracle",
        "sample": f"FP64 oracle, {K} passes (step + retract) of the headline workload on the whole "
                  f"{A32.shape[0]} x {A32.shape[1]} matrix from its default start, {allt} threads",
        "single_thread_iters_per_s": v_one,
        "single_unit_5000x50000_SL1_f0.05": {"passes": K2, "iters_per_s_all_threads": c2_all,
                                             "iters_per_s_one_thread": c2_one},
        "small_100x1000_SL1_converged": {"solves_per_s": 1.0 / c1_s, "passes": r1["n_iter"],
                                         "threads": allt},
        "host": host_info(),
    }


# Panels of the efficiency experiment (Section 4.1, Fig. 3 a-d): form and gamma
# (a fraction of max ||a_i||, squared for the l0 forms).
SWEEP_PANELS = (("SL0", 1, 0.01), ("BL0", 3, 0.01), ("SL1", 0, 0.05), ("BL1", 2, 0.05))
SWEEP_SIZES = (500, 1000, 2000, 4000, 8000, 16000, 32000)


def oracle_threads() -> int:
    import oracle as O
    return O.num_threads()


def sweep_cpu_baseline(mats, fid, m, gam, budget_s):
    """CPU baseline of the sweep: the FP64 oracle's solve of the first instances
    on the host's cores while `budget_s` lasts; returns the times (s)."""
    import oracle as O
    ot = []
    spent = 0.0
    for a in mats:
        A64 = a.astype(np.float64)
        g = gam(a)
        t = time.perf_counter()
        if fid < 2:
            O.solve_deflated(A64, fid, m, g)
        else:
            O.solve(A64, fid, m, g)
        el = time.perf_counter() - t
        ot.append(el)
        spent += el
        if spent + el > budget_s:
            break
    return ot


def sweep_parity(G, a, d, fid, m, g, passes=8):
    """Fixed-pass comparison of one instance with the oracle: the GPU and the
    FP64 oracle both run `passes` passes per component (tol = 0) from their
    default starts; largest relative 2-norm error of x and z over the
    components, largest relative error of the final objective, and the number
    of support memberships that differ."""
    import oracle as O
    A64 = a.astype(np.float64)
    if fid < 2:
        r = G.solve_deflated(d, fid, m, g, tol=0.0, max_iter=passes)
        ref = O.solve_deflated(A64, fid, m, g, tol=0.0, max_iter=passes)
        F, Fo = [t[-1] for t in r.traces], [t[-1] for t in ref["traces"]]
    else:
        r = G.solve(d, fid, m, g, tol=0.0, max_iter=passes)
        ref = O.solve(A64, fid, m, g, tol=0.0, max_iter=passes)
        F, Fo = [r.trace[-1]], [ref["trace"][-1]]
    X = r.X.cpu().numpy().astype(np.float64)
    Z = r.Z.cpu().numpy().astype(np.float64)
    sup = r.support_mask().cpu().numpy()
    ex = max(float(np.linalg.norm(X[:, j] - ref["X"][:, j]) / np.linalg.norm(ref["X"][:, j]))
             for j in range(m))
    ez = max(float(np.linalg.norm(Z[:, j] - ref["Z"][:, j]) / max(np.linalg.norm(ref["Z"][:, j]), 1e-300))
             for j in range(m))
    eF = max(abs(x - y) / max(abs(y), 1e-300) for x, y in zip(F, Fo))
    return {"passes": passes, "x": ex, "z": ez, "F": float(eF),
            "support_diff": int((sup != ref["support"]).sum())}


def sweep(args):
    """Average time per solve over `--sweep-seeds` instances per size, m = 5
    components, N(0,1) matrices (the paper does not state the distribution),
    default start, tol = 1e-4, at most 1000 passes.  The single-unit panels
    compute their 5 components by deflation, the block panels solve one block of
    5.  A is resident on the device; the time covers the whole solve call
    (start, passes, finalize, copy of the traces to the host).  The FP64 oracle
    runs the same solves on the host on the first instances, within a budget,
    and the first instance of each cell is compared with it at a fixed pass
    count (sweep_parity)."""
    import torch
    import paper_1312_6182_amd as G
    from workloads import generators as W

    G.load()
    m = 5
    rows = []
    oracle_stopped = {name: False for name, _, _ in SWEEP_PANELS}
    last_oracle = {name: 0.0 for name, _, _ in SWEEP_PANELS}
    for N in SWEEP_SIZES:
        P = N // 10
        mats = [W.gaussian(P, N, 9000 + 97 * N + s) for s in range(args.sweep_seeds)]
        devs = [torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t() for a in mats]
        torch.cuda.synchronize()
        for name, fid, frac in SWEEP_PANELS:
            l0 = fid in (1, 3)

            def gam(a):
                c = column_norm_max(a)
                return frac * (c * c if l0 else c)

            def run(d, g):
                if fid < 2:
                    r = G.solve_deflated(d, fid, m, g)
                    return r, sum(r.n_iter), [t[-1] for t in r.traces]
                r = G.solve(d, fid, m, g)
                return r, r.n_iter, [r.trace[-1]]

            run(devs[0], gam(mats[0]))  # plan, code objects
            torch.cuda.synchronize()
            times, passes, finals = [], [], []
            for a, d in zip(mats, devs):
                g = gam(a)
                t = time.perf_counter()
                _, npass, fin = run(d, g)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
                passes.append(npass)
                finals.append(fin)
            row = {"N": N, "P": P, "panel": name, "gamma_frac": frac, "instances": len(mats),
                   "gpu_ms": 1e3 * float(np.mean(times)), "gpu_ms_max": 1e3 * float(np.max(times)),
                   "passes_mean": float(np.mean(passes))}
            if not oracle_stopped[name] and last_oracle[name] * 4.5 <= args.sweep_oracle_seconds:
                ot = sweep_cpu_baseline(mats, fid, m, gam, args.sweep_oracle_seconds)
                last_oracle[name] = float(np.mean(ot))
                row["parity_vs_oracle"] = sweep_parity(G, mats[0], devs[0], fid, m, gam(mats[0]))
            else:
                ot = []
                oracle_stopped[name] = True
            if ot:
                row.update({"oracle_ms": 1e3 * float(np.mean(ot)), "oracle_instances": len(ot),
                            "oracle_threads": oracle_threads(),
                            "ratio_oracle_over_gpu": float(np.mean(ot)) / float(np.mean(times))})
            rows.append(row)
            print(f"[sweep] {json.dumps(row)}", file=sys.stderr, flush=True)
        del devs
        torch.cuda.empty_cache()
    print(json.dumps({"sweep": "Section 4.1 efficiency experiment, P = N/10, m = 5",
                      "data": "synthetic N(0,1)", "rows": rows}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    import torch
    import paper_1312_6182_amd as G
    from workloads import generators as W

    G.load()
    form_id = {"SL1": 0, "SL0": 1, "BL1": 2, "BL0": 3}[args.form]
    l0 = form_id in (1, 3)
    m = 1 if form_id < 2 else args.m
    frac = args.frac if args.frac is not None else (0.01 if l0 else 0.05)
    t = time.perf_counter()
    planted = max(1, min(args.m, 64))
    A32, _, _ = W.planted_block(args.p, args.n, planted, args.seed, k=200)
    cmax = column_norm_max(A32)
    gamma = frac * (cmax * cmax if l0 else cmax)
    At = torch.from_numpy(np.ascontiguousarray(A32.T)).cuda()
    Ad = At.t()
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t
    print(f"[bench] data ready in {prep_s:.1f}s: p={args.p} n={args.n} m={m} {args.form} "
          f"gamma={gamma:.4g}", file=sys.stderr, flush=True)

    tuned = None
    if not args.no_autotune:
        tuned = G.autotune(Ad, form_id, m, gamma, passes=3)
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
    r, ms, kms, launches, kname = time_gpu(G, torch, Ad, form_id, m, gamma, args.steps, args.warmup)
    ms_per_step = ms / args.steps
    iters_per_s = 1000.0 / ms_per_step
    a_bytes = float(args.p) * args.n * 4.0
    alg_bytes = algorithmic_bytes(kname, args.p, args.n, m)
    k_avg_ms = kms / max(1, launches)
    achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
    nnz = int(r.support_mask().sum().item())
    print(f"[bench] {args.steps} passes in {ms:.2f} ms; {kname} avg {k_avg_ms*1e3:.1f} us "
          f"({achieved:.0f} GB/s); final support {nnz}", file=sys.stderr, flush=True)
    wkey = f"{args.form}_m{m}_p{args.p}_n{args.n}"
    traffic = traffic_from_profiles(kname, wkey)

    out = {
        "metric": METRIC,
        "value": iters_per_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.form} m={m}, A {args.p}x{args.n} FP32 column-major (N(0,1) noise + "
                        f"{planted} planted 200-sparse components, seed {args.seed}), "
                        f"gamma={frac} max||a_i||{'^2' if l0 else ''}, mu=1, tol=0 (fixed passes)",
            "p": args.p, "n": args.n, "m": m, "form": args.form, "gamma": gamma,
            "kernel_config": tuned["choice"] if tuned else "default",
        },
        "a_stream_gbps_whole_step": a_bytes * args.steps / (ms * 1e-3) / 1e9,
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_us": k_avg_ms * 1e3,
            "timed_launches": launches,
        },
        "final_support_nnz": nnz,
    }
    if args.c4_only:
        i0 = int(np.argmax(np.einsum("ij,ij->j", A32, A32, dtype=np.float64)))
        x0 = A32[:, [i0]].astype(np.float64)
        x0 = (x0 / np.linalg.norm(x0)).astype(np.float32).astype(np.float64)
        out["c4_gamma_path"], _ = gamma_path_leg(G, torch, W, Ad, A32, cmax, x0)
        if args.copy_calibration_mib > 0:
            copy_calibration(torch, args.copy_calibration_mib)
        print(json.dumps(out))
        return
    if not args.no_extra:
        extra = {}
        # at least 33 timed passes per leg whatever --steps is, so that every
        # leg's figure is a per-pass rate, not the one-off start of its solve
        xs = max(33, args.steps // 3)

        def rec(name, Adev, fid, mm, g, mu=None):
            r2, ms2, kms2, l2, kn2 = time_gpu(G, torch, Adev, fid, mm, g, xs, 2, mu=mu)
            pp, nn = Adev.shape
            extra[name] = {"iters_per_s": 1000.0 * xs / ms2, "kernel": kn2,
                           "kernel_gbps": algorithmic_bytes(kn2, pp, nn, mm)
                           / (kms2 / max(1, l2) * 1e-3) / 1e9,
                           "ms_per_step": ms2 / xs}
            if mm > 1:
                live = int(r2.support_mask().any(dim=0).sum().item())
                extra[name]["dead_components"] = mm - live
                extra[name]["kernel_tflops"] = 2.0 * pp * nn * mm / (kms2 / max(1, l2) * 1e-3) / 1e12
            print(f"[bench] extra {name}: {extra[name]}", file=sys.stderr, flush=True)

        if args.p == 10000 and args.n == 100000:
            inv8 = list(1.0 / np.arange(1, 9))
            rec("c3_BL0_m8", Ad, 3, 8, 0.01 * cmax * cmax)
            rec("c3_BL1_m8_mu_inv", Ad, 2, 8, 0.05 * cmax, mu=inv8)
            rec("c3_BL0_m8_mu_inv", Ad, 3, 8, 0.01 * cmax * cmax, mu=inv8)
            rec("c3_SL1_m1", Ad, 0, 1, 0.05 * cmax)
            rec("c3_BL1X_m8", Ad, 4, 8, 0.05 * cmax)
            extra["c3_SL1_deflated_5"] = deflated_leg(G, torch, Ad, 0.05 * cmax, xs)
            print(f"[bench] extra c3_SL1_deflated_5: {extra['c3_SL1_deflated_5']}", file=sys.stderr,
                  flush=True)
            # m = 64 on the matrix with 64 planted components (beta_j = 5 sqrt(n)/j)
            A64p, _, _ = W.planted_block(args.p, args.n, 64, args.seed, k=200)
            c64 = column_norm_max(A64p)
            A64d = torch.from_numpy(np.ascontiguousarray(A64p.T)).cuda().t()
            del A64p
            inv64 = list(1.0 / np.arange(1, 65))
            if not args.no_autotune:
                G.autotune(A64d, 2, 64, 0.05 * c64, passes=2)
            rec("c3_BL1_m64", A64d, 2, 64, 0.05 * c64)
            rec("c3_BL0_m64", A64d, 3, 64, 0.01 * c64 * c64)
            rec("c3_BL1_m64_mu_inv", A64d, 2, 64, 0.05 * c64, mu=inv64)
            rec("c3_BL0_m64_mu_inv", A64d, 3, 64, 0.01 * c64 * c64, mu=inv64)
            del A64d
            torch.cuda.empty_cache()
        A2, _, _, _ = W.planted_single(5000, 50000, args.seed, k=500)
        c2max = column_norm_max(A2)
        A2d = torch.from_numpy(np.ascontiguousarray(A2.T)).cuda().t()
        rec("c2_SL1_f0.05", A2d, 0, 1, 0.05 * c2max)
        rec("c2_SL0_f0.01", A2d, 1, 1, 0.01 * c2max * c2max)
        rec("c2_SL1_f0.01_dense", A2d, 0, 1, 0.01 * c2max)
        del A2d
        out["extra"] = extra
    kept = None
    if not args.no_extra and args.p == 10000 and args.n == 100000:
        i0 = int(np.argmax(np.einsum("ij,ij->j", A32, A32, dtype=np.float64)))
        x0 = A32[:, [i0]].astype(np.float64)
        x0 = (x0 / np.linalg.norm(x0)).astype(np.float32).astype(np.float64)
        out["c4_gamma_path"], kept = gamma_path_leg(G, torch, W, Ad, A32, cmax, x0)
    if not args.no_extra and args.serve_requests > 0:
        del Ad, At
        torch.cuda.empty_cache()
        out["c5_serving"] = serving_leg(W, args.serve_requests, args.serve_pmax, args.serve_nmax,
                                        args.serve_repeat, args.serve_arena_gb)
    if kept is not None and not args.no_accuracy:
        print("[bench] gamma path accuracy against the FP64 oracle", file=sys.stderr, flush=True)
        out["c4_gamma_path"]["accuracy"] = gamma_path_accuracy(A32, x0, kept)
    if args.copy_calibration_mib > 0:
        copy_calibration(torch, args.copy_calibration_mib)
    if not args.no_cpu:
        print("[bench] timing the oracle on host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(A32, form_id, m, gamma)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
