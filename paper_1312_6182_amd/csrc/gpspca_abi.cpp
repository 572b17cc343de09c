// C ABI of the gfx950 GP-SPCA library: argument validation, workspace layout,
// kernel selection and the iteration driver.
//
// Per pass k (Section 2, Table 1):
//   m = 1, p <= 20480   k_pass_m1 (one read of A; correlation, threshold and
//                       back-projection fused)
//   otherwise           k_corr (correlation + threshold, one read of A) and
//                       k_backproj (reads only the columns in the support)
//   then                k_reduce_partials -> k_gram -> k_stop -> k_apply
//                       (after k_pass_m1: k_reduce_m1 -> k_stop_x1, which
//                       writes x_{k+1} itself)
// The stopping rule runs on the device; the host polls the control block once
// per chunk of passes and never per pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "gpspca_internal.h"

namespace gpspca {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define GPSPCA_HIP(expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(GPSPCA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// GPSPCA_MFMA_BALANCE=0 turns the balanced partition of the matrix-core
// correlation off (every wave then takes whole tiles only).
static bool mfma_balance_enabled() {
    const char* e = std::getenv("GPSPCA_MFMA_BALANCE");
    return !(e && e[0] == '0');
}

// ---------------------------------------------------------------- device info
static int device_cus(int* out) {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    GPSPCA_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0 || dev >= 64) return fail(GPSPCA_EDEVICE, "device index out of range");
    if (cached[dev] == 0) {
        int cus = 0;
        GPSPCA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        cached[dev] = cus > 0 ? cus : 1;
    }
    *out = cached[dev];
    return GPSPCA_OK;
}

// ----------------------------------------------------------------- validation
static int check_matrix(const gpspca_matrix* A) {
    if (!A) return fail(GPSPCA_EINVAL, "A is NULL");
    if (!A->data) return fail(GPSPCA_EINVAL, "A->data is NULL");
    if (A->p < 1 || A->n < 1) return fail(GPSPCA_EINVAL, "p and n must be >= 1");
    if (A->p > (int64_t)1 << 30) return fail(GPSPCA_EINVAL, "p must be <= 2^30");
    if (A->lda < A->p) return fail(GPSPCA_EINVAL, "lda must be >= p");
    if (A->n >= ((int64_t)1 << 31)) return fail(GPSPCA_EINVAL, "n must be < 2^31");
    switch (A->dtype) {
        case GPSPCA_F32:
            if (A->col_scale)
                return fail(GPSPCA_EINVAL, "col_scale applies to BF16 / F8E4M3 storage only");
            break;
        case GPSPCA_BF16:
        case GPSPCA_F8E4M3: {
            const int64_t q = A->dtype == GPSPCA_BF16 ? 8 : 16;
            if (A->lda % q != 0)
                return fail(GPSPCA_EINVAL, "lda of BF16 (F8E4M3) storage must be a multiple of 8 (16)");
            if ((reinterpret_cast<uintptr_t>(A->data) & 15) != 0)
                return fail(GPSPCA_EINVAL, "BF16 / F8E4M3 data must be 16-byte aligned");
            if (A->dtype == GPSPCA_F8E4M3 && !A->col_scale)
                return fail(GPSPCA_EINVAL, "F8E4M3 storage needs col_scale");
            break;
        }
        default:
            return fail(GPSPCA_EDTYPE, "unknown dtype");
    }
    return GPSPCA_OK;
}

int check_problem(const gpspca_matrix* A, int form, int m, double gamma, const double* mu) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (form < GPSPCA_SL1 || form > GPSPCA_BL0) return fail(GPSPCA_EINVAL, "unknown formulation");
    const bool block = form >= GPSPCA_BL1;
    if (!block && m != 1) return fail(GPSPCA_EINVAL, "single-unit formulations need m = 1");
    if (m < 1 || m > A->p) return fail(GPSPCA_EINVAL, "need 1 <= m <= p");
    if (m > kMaxM) return fail(GPSPCA_EINVAL, "m exceeds GPSPCA_MAX_M");
    if (!std::isfinite(gamma) || gamma < 0.0) return fail(GPSPCA_EINVAL, "gamma must be finite and >= 0");
    if (block && mu) {
        for (int j = 0; j < m; ++j)
            if (!std::isfinite(mu[j]) || !(mu[j] > 0.0))
                return fail(GPSPCA_EINVAL, "mu must be finite and > 0");
    }
    return GPSPCA_OK;
}

// ------------------------------------------------------------------ tuning
// Configurations chosen by gpspca_autotune, per (storage, m, p, n, vector
// alignment, gamma path); consulted by every plan after the environment
// overrides (GPSPCA_CORR_KERNEL, GPSPCA_MFMA_STAGES, GPSPCA_MFMA_WAVES_PER_CU).
struct TuneKey {
    int dtype, m, vec, path;
    int64_t p, n;
    bool operator<(const TuneKey& o) const {
        return std::tie(dtype, m, vec, path, p, n) < std::tie(o.dtype, o.m, o.vec, o.path, o.p, o.n);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, Tune> g_tune;

static TuneKey tune_key(const gpspca_matrix* A, int m, int path) {
    const int vec = ((A->lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(A->data) & 15) == 0);
    return TuneKey{A->dtype, m, vec, path, A->p, A->n};
}

static bool tune_lookup(const TuneKey& k, Tune* t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

static Tune env_tune() {
    Tune t{kTuneDefault, 0, 0};
    if (const char* f = std::getenv("GPSPCA_CORR_KERNEL")) {
        const std::string fk = f;
        t.kernel = fk == "mfma" ? kTuneMfma : fk == "vx" ? kTuneVx : fk == "valu" ? kTuneValu
                 : fk == "rd" ? kTuneRd : fk == "rd128" ? kTuneRd128 : fk == "wg" ? kTuneWg
                 : fk == "x3" ? kTuneX3 : fk == "qw" ? kTuneQw
                 : fk == "mv" ? -1 : kTuneDefault;
    }
    if (const char* e = std::getenv("GPSPCA_MFMA_STAGES")) t.stages = std::atoi(e);
    if (const char* e = std::getenv("GPSPCA_MFMA_WAVES_PER_CU")) t.waves = std::atoi(e);
    return t;
}

// Active fraction (in 1/1024) of the n columns from which a pass is
// back-projected densely on the matrix cores.  The support-restricted kernel
// reads each active column once per group of 16 components; the dense one
// reads every column once for all components.  The thresholds are the measured
// crossovers on a 10000 x 100000 matrix (gamma paths and block solves with
// 16 to 64 components at 2% to 55% activity), per storage type and number of
// component groups (1, 2, 3, 4); for FP32 they are near 0.40, 0.22, 0.19 and
// 0.18.  Frozen-support passes visit only listed columns and leave S of the
// others unwritten, so they stay sparse.
static int backproj_threshold(const gpspca_matrix* A, int m, int vec4, int restricted) {
    const int never = 2 * 1024;
    if (restricted || m <= 4 || A->p < 64 || (A->dtype == GPSPCA_F32 && !vec4)) return never;
    if (const char* e = std::getenv("GPSPCA_BACKPROJ")) {
        const std::string v = e;
        if (v == "dense") return 0;
        if (v == "sparse") return never;
        if (!v.empty() && v != "auto") return std::max(0, std::min(never, std::atoi(e)));
    }
    static const int thr[3][4] = {{410, 225, 195, 185},    // FP32
                                  {185, 125, 110, 100},    // bfloat16
                                  {195, 135, 125, 120}};   // e4m3
    const int st = A->dtype == GPSPCA_BF16 ? 1 : A->dtype == GPSPCA_F8E4M3 ? 2 : 0;
    const int groups = std::min(4, (m + 15) / 16);
    return thr[st][groups - 1];
}

// ----------------------------------------------------------------------- plan
static void make_plan(const gpspca_matrix* A, int form, int m, int max_iter, int ncu, Plan* pl,
                      int path = 0, int restricted = 0, const Tune* force = nullptr) {
    std::memset(pl, 0, sizeof(Plan));
    pl->path = path;
    pl->restricted = restricted;
    pl->dtype = A->dtype;
    pl->p = A->p;
    pl->n = A->n;
    pl->lda = A->lda;
    pl->m = m;
    pl->form = form;
    pl->l0 = (form == GPSPCA_SL0 || form == GPSPCA_BL0) ? 1 : 0;
    pl->max_iter = max_iter;
    // rows of the internal X buffers: room for the 32-row stages of the matrix-core
    // kernel and at least one quad of zero rows past p
    pl->ldx = (int)align_up((size_t)A->p + 4, 32);
    pl->vec4 = ((A->lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(A->data) & 15) == 0);
    const int64_t nq = cdiv(A->p, 4);
    const bool f32 = A->dtype == GPSPCA_F32;

    pl->fused_m1 = (m == 1 && A->p <= 20480 && !path && f32 && !restricted) ? 1 : 0;
    if (pl->fused_m1) {
        const int cand[4] = {64, 256, 512, 1024};
        int T = 1024;
        for (int c : cand)
            if (cdiv(nq, c) <= 5) { T = c; break; }
        pl->m1_threads = T;
        pl->m1_kq = (int)std::max<int64_t>(1, cdiv(nq, T));
        const int per_cu = T <= 64 ? 8 : T <= 256 ? 2 : 1;
        int64_t grid = (int64_t)ncu * per_cu;
        grid = std::min<int64_t>(grid, std::max<int64_t>(1, A->n / 8));
        pl->m1_grid = (int)std::max<int64_t>(1, grid);
        pl->npart = pl->m1_grid;
        pl->nwave_part = pl->m1_grid;
    } else {
        // correlation kernel.  Choice: an explicit configuration (the autotuner
        // trying candidates), else the environment (tests, benchmarks), else the
        // autotuner's table, else the measured default -- register-resident X
        // for m <= 4, the FP32 matrix cores up to m = 32, and the FP32 values
        // split into bfloat16 parts on the bfloat16 matrix cores beyond (m = 64
        // on 10000 x 100000: 1243 us against 1301 for the best FP32 kernel).
        Tune tn{kTuneDefault, 0, 0};
        if (force) {
            tn = *force;
        } else if (!restricted) {
            tn = env_tune();
            Tune tt;
            if (tn.kernel == kTuneDefault && tn.stages == 0 && tn.waves == 0 &&
                tune_lookup(tune_key(A, m, path), &tt))
                tn = tt;
        }
        const bool vx_ok = f32 && pl->vec4 && m >= 2 && m <= 8 && A->p <= 10240 && A->p >= 4 && !path;
        const bool mv_ok = f32 && pl->vec4 && m <= 16 && A->p >= 4;
        if (restricted) {}
        else if (!f32) pl->use_q = 1;
        else if (tn.kernel == -1 && mv_ok) pl->use_mv = 1;
        else if (tn.kernel == kTuneVx && vx_ok) pl->use_vx = 1;
        else if (tn.kernel == kTuneMfma && pl->vec4) pl->use_mfma = 1;
        else if (tn.kernel == kTuneRd && pl->vec4) pl->use_mfma = pl->use_rd = 1;
        else if (tn.kernel == kTuneRd128 && pl->vec4) pl->use_mfma = pl->use_rd = pl->rd128 = 1;
        else if (tn.kernel == kTuneX3 && pl->vec4) pl->use_mfma = pl->use_x3 = 1;
        else if (tn.kernel == kTuneWg && pl->vec4) pl->use_mfma = pl->use_wg = 1;
        else if (tn.kernel == kTuneValu) {}
        else if (vx_ok && m <= 4) pl->use_vx = 1;
        else if (m > 32 && pl->vec4) pl->use_mfma = pl->use_x3 = 1;   // FP32 matrix cores are the bound
        else pl->use_mfma = pl->vec4;
        if (pl->use_q && tn.kernel != kTuneMfma) {
            // 16/8-bit storage, four-wave workgroups sharing X (the default): one
            // per CU.  Staging: 2 stages of up to 8 tiles per wave, 3 stages of
            // 4 tiles (stages = 3), or for e4m3 2 stages of 4 tiles (stages = 2)
            pl->use_qw = 1;
            pl->corr_M = 16;
            pl->mfma_stages = (tn.stages == 2 || tn.stages == 3) ? tn.stages : 8;
            pl->waves_per_cu = 4;
            const int64_t grid = std::min<int64_t>(ncu, cdiv(cdiv(A->n, 16), 4));
            pl->corr_grid = (int)std::max<int64_t>(1, grid);
            pl->nwave_part = pl->corr_grid * 4;
        } else if (pl->use_q) {
            // 16/8-bit storage: bfloat16 matrix cores, one wavefront per workgroup
            pl->corr_M = 16;
            pl->mfma_stages = corr_q_stages(A->dtype, m, tn.stages);
            const int fit = corr_q_blocks_per_cu(A->dtype, m, pl->mfma_stages);
            pl->waves_per_cu = std::min(fit, tn.waves > 0 ? tn.waves : 4);
            int64_t grid = std::min<int64_t>((int64_t)ncu * pl->waves_per_cu, cdiv(A->n, 16));
            pl->corr_grid = (int)std::max<int64_t>(1, grid);
            pl->nwave_part = pl->corr_grid;
        } else if (pl->use_vx) {
            // X rows in registers: one workgroup per CU (512 threads) or two (256)
            pl->corr_M = m <= 2 ? 2 : m <= 4 ? 4 : 8;
            pl->vx_threads = (cdiv(nq, 256) <= 5) ? 256 : 512;
            pl->vx_kq = (int)std::max<int64_t>(1, cdiv(nq, pl->vx_threads));
            const int per_cu = pl->vx_threads == 256 ? 2 : 1;
            int64_t grid = std::min<int64_t>((int64_t)ncu * per_cu, std::max<int64_t>(1, A->n / 4));
            pl->corr_grid = (int)std::max<int64_t>(1, grid);
            pl->nwave_part = pl->corr_grid;
        } else if (pl->use_mfma || pl->use_mv) {
            // one wavefront per workgroup; 4 per CU by default (a fifth wave per
            // CU, or a sixth, was measured slower), never more than LDS allows
            pl->corr_M = 16;
            // m <= 16: 2, 3 or 4 stages of 4 tiles, or "8": 2 stages of 8 tiles
            // (the default: a wave's columns then fit one chunk, so X is staged
            // once per wave -- measured 3.5% faster than 4 stages of 4 tiles);
            // m <= 32: 3 stages of 4 tiles, or "8" (the default, 7.6% faster at
            // m = 32: half the X instructions per byte of A)
            pl->mfma_stages = (m <= 16) ? (((tn.stages >= 2 && tn.stages <= 4) || tn.stages == 8)
                                               ? tn.stages : 8)
                            : (m <= 32) ? (tn.stages == 3 ? 3 : 8)
                                        : 2;
            pl->rd_depth = (tn.stages == 2 || tn.stages == 3 || tn.stages == 6) ? tn.stages : 4;
            int per_cu = tn.waves > 0 ? tn.waves : 4;
            if (pl->use_x3) pl->rd_depth = tn.stages == 3 ? 3 : 2;
            if (!pl->use_rd && !pl->use_mv && !pl->use_x3)
                per_cu = std::min(per_cu, corr_mfma_blocks_per_cu(m, pl->mfma_stages));
            if (pl->use_mv) per_cu = 4;
            pl->waves_per_cu = per_cu;
            int64_t grid = std::min<int64_t>((int64_t)ncu * per_cu, cdiv(A->n, 16));
            pl->corr_grid = (int)std::max<int64_t>(1, grid);
            pl->nwave_part = pl->corr_grid;
            if (pl->use_wg) {
                // one four-wave workgroup per CU (the LDS of a CU holds its stages)
                if (m > 16) pl->mfma_stages = 8;
                pl->waves_per_cu = 4;
                grid = std::min<int64_t>((int64_t)ncu, cdiv(cdiv(A->n, 16), 4));
                pl->corr_grid = (int)std::max<int64_t>(1, grid);
                pl->nwave_part = pl->corr_grid * 4;
            }
        } else {
            pl->corr_M = m >= 5 ? 8 : m >= 3 ? 4 : m == 2 ? 2 : 1;
            int64_t grid = std::min<int64_t>((int64_t)ncu * 2, std::max<int64_t>(1, cdiv(A->n, 32)));
            pl->corr_grid = (int)std::max<int64_t>(1, grid);
            pl->nwave_part = pl->corr_grid * 4;
        }
        pl->bp_kq = 2;
        pl->bp_rb = (int)cdiv(nq, 256 * pl->bp_kq);
        // column ranges of >= 1024 columns, about 4 workgroups per CU in all; a
        // matrix too small to give every CU a workgroup that way takes ranges of
        // >= 128 columns instead, and a smaller one still ranges of >= 32 up to
        // 128 ranges (each workgroup walks its range's active columns in
        // dependent batches, so long ranges are latency-bound; 128 partials
        // still take the fused reduction)
        const int64_t want = std::max<int64_t>(1, (4LL * ncu) / pl->bp_rb);
        int64_t cr = std::min<int64_t>(cdiv(A->n, 1024), want);
        if (cr * pl->bp_rb < ncu) cr = std::min<int64_t>(cdiv(A->n, 128), want);
        if (cr * pl->bp_rb < ncu)
            cr = std::min<int64_t>(std::min<int64_t>(cdiv(A->n, 32), want), std::max<int64_t>(cr, 128));
        pl->bp_cr = (int)std::max<int64_t>(1, cr);
        pl->npart = pl->bp_cr;
        pl->bp_thr = backproj_threshold(A, m, pl->vec4, restricted);
        // the decision needs the pass's active-column count, which only the
        // correlation kernels below keep
        if (!(pl->use_mfma || pl->use_vx || pl->use_mv || pl->use_q)) pl->bp_thr = 2 * 1024;
    }
    // columns of the X buffers: the matrix-core kernels (corr_M = 16) read every
    // column of their 1, 2 or 4 groups of 16 (components past m are zero)
    pl->mpad = pl->fused_m1 ? 1
             : pl->corr_M == 16 ? 16 * (m <= 16 ? 1 : m <= 32 ? 2 : 4)
             : (int)align_up((size_t)m, (size_t)pl->corr_M);
    // interleaved copies of X (FP32 row quads) for the matrix-core kernels
    pl->xil_bytes = (pl->use_mfma || pl->use_q) ? 4 * (size_t)pl->ldx * (size_t)pl->mpad : 0;
    const int64_t ne = (int64_t)m * pl->ldx;
    const int64_t bx = cdiv(ne, 256);
    int64_t split = cdiv(2LL * ncu, bx);
    split = std::min<int64_t>(split, std::max<int64_t>(1, pl->npart / 8));
    split = std::min<int64_t>(split, 64);
    pl->red_split = (int)std::max<int64_t>(1, split);
    // row blocks of the Gram products: 256 rows, 128 when the LDS tile would
    // not fit, and (m > 1) 64 when 128-row blocks would leave CUs without one
    pl->gram_rows = ((size_t)(m + 1) * 256 * 16 <= 140000) ? 256 : 128;
    if (m > 1 && cdiv(A->p, 128) < ncu) pl->gram_rows = 64;
    pl->gram_grid = (int)cdiv(A->p, pl->gram_rows);
    // the fused m = 1 pass leaves one partial per workgroup (hundreds), and
    // small matrices take many short column ranges: hundreds of partials are
    // summed faster by the split reduction, whose grid also spans the partials
    pl->fused_gram = (m <= 16 && !pl->fused_m1 && pl->npart <= 128) ? 1 : 0;
    pl->gram_blocks = pl->fused_gram ? (int)cdiv(A->p, 64)
                      : pl->fused_m1 ? (int)cdiv(A->p, kRm1Rows)
                                     : pl->gram_grid;
    // 256 / m support words (32 columns each) per finalize workgroup
    pl->fin_grid = (int)std::max<int64_t>(1, cdiv(cdiv(A->n, 32), 256 / std::max(1, m)));
    pl->topm_grid = (int)std::max<int64_t>(1, std::min<int64_t>(256, cdiv(A->n, 1024)));

    // balanced partition of the FP32 matrix-core correlation (2 stages of 8
    // tiles, one or two component groups): when the waves do not divide the tiles,
    // each takes q whole tiles and an equal row share of the leftover ones
    pl->bal = pl->bal_q = pl->bal_rem = 0;
    if (pl->use_mfma && !pl->use_rd && !pl->use_x3 && !pl->use_wg && !pl->use_mv &&
        !pl->use_q && !pl->use_qw && !pl->use_vx && !pl->fused_m1 && !pl->restricted &&
        m <= 32 && pl->mfma_stages == 8 && A->p >= 64 && mfma_balance_enabled()) {
        const int64_t ntile = cdiv(A->n, 16), W = pl->corr_grid;
        const int64_t q = ntile / W, rem = ntile % W;
        if (rem > 0 && q >= 1 && q + 1 <= 8) {
            pl->bal = 1;
            pl->bal_q = (int)q;
            pl->bal_rem = (int)rem;
            pl->nwave_part = (int)(W + rem);
        }
    }

    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1), 256);
        return at;
    };
    const size_t P = (size_t)A->p, N = (size_t)A->n, M = (size_t)m, L = (size_t)pl->ldx;
    pl->o_ctrl = take(sizeof(Ctrl));
    pl->o_trace = take(sizeof(double) * (size_t)std::max(1, max_iter) * (path ? M : 1));
    pl->o_x0 = take(sizeof(float) * L * (size_t)pl->mpad);
    pl->o_x1 = take(sizeof(float) * L * (size_t)pl->mpad);
    pl->o_s = take(sizeof(float) * N * M);
    pl->o_act = take(N);
    pl->o_gpart = take(sizeof(float) * (size_t)pl->npart * M * L);
    pl->o_touched = take(sizeof(int) * (size_t)pl->npart);
    pl->o_fpart = take(sizeof(double) * (size_t)pl->nwave_part * M);
    pl->o_nnzpart = take(sizeof(int) * (size_t)pl->nwave_part * M);
    pl->o_l1 = take(sizeof(double) * (size_t)pl->red_split * M * L);
    pl->o_g64 = take(sizeof(double) * M * P);
    pl->o_gram = take(sizeof(double) * (size_t)std::max(pl->gram_grid, pl->gram_blocks) * 3 * M * M);
    pl->o_coef = take(sizeof(double) * 6 * M * M);  // Omega, Psi, G^T G, G^T X, X^T X, V
    pl->o_norms = take(sizeof(double) * N);
    pl->o_cand_v = take(sizeof(double) * (size_t)pl->topm_grid * M);
    pl->o_cand_i = take(sizeof(int64_t) * (size_t)pl->topm_grid * M);
    pl->o_idx = take(sizeof(int64_t) * M);
    pl->o_fin = take(sizeof(double) * (size_t)pl->fin_grid * M);
    pl->o_invn = take(sizeof(double) * M);
    pl->o_fcomp = take(sizeof(double) * 2 * M);
    pl->o_pstate = take(path ? sizeof(PathState) * M : 1);
    pl->o_list = take(sizeof(int) * (N + 64));  // frozen-support column list + its count
    const bool xil = pl->use_mfma || pl->use_q;   // interleaved copies of X for the DMA kernels
    pl->o_xil0 = take(xil ? pl->xil_bytes : 1);
    pl->o_xil1 = take(xil ? pl->xil_bytes : 1);
    pl->o_fsum = take(sizeof(double) * 2 * M);   // per-component objective and support sums
    pl->o_xpart = take(pl->bal ? sizeof(float) * 512 * (size_t)(m <= 16 ? 1 : 2) * pl->corr_grid : 1);
    pl->total = o;
}

// Configurations the autotuner tries for this problem (the default first).
static std::vector<Tune> tune_candidates(const gpspca_matrix* A, int m, int path) {
    std::vector<Tune> c;
    c.push_back(Tune{kTuneDefault, 0, 0});
    const bool vec = ((A->lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(A->data) & 15) == 0);
    if (A->dtype != GPSPCA_F32) {
        c.push_back(Tune{kTuneQw, 3, 0});
        if (A->dtype == GPSPCA_F8E4M3) c.push_back(Tune{kTuneQw, 2, 0});
        c.push_back(Tune{kTuneMfma, 2, 4});
        c.push_back(Tune{kTuneMfma, 3, 4});
        c.push_back(Tune{kTuneMfma, 8, 4});
        return c;
    }
    if (m == 1 && !path && A->p <= 20480) return c;  // the fused single-unit pass
    if (!vec) return c;
    if (m <= 16) {
        for (int st = 2; st <= 4; ++st) c.push_back(Tune{kTuneMfma, st, 4});
        c.push_back(Tune{kTuneMfma, 8, 4});   // 2 stages of 8-tile chunks
        c.push_back(Tune{kTuneMfma, 2, 8});
        c.push_back(Tune{kTuneWg, 8, 4});
        c.push_back(Tune{kTuneWg, 4, 4});
    } else {
        c.push_back(Tune{kTuneMfma, 0, 4});
        if (m <= 32) c.push_back(Tune{kTuneMfma, 3, 4});
        c.push_back(Tune{kTuneWg, 8, 4});
    }
    if (m > 16) {
        c.push_back(Tune{kTuneX3, 2, 4});
        c.push_back(Tune{kTuneX3, 3, 4});
    }
    c.push_back(Tune{kTuneRd, 4, 4});
    c.push_back(Tune{kTuneRd128, 4, 4});
    c.push_back(Tune{kTuneRd128, 3, 4});
    if (m >= 2 && m <= 8 && A->p <= 10240 && !path) c.push_back(Tune{kTuneVx, 0, 0});
    return c;
}

// Workspace that every configuration of the problem fits in (tuned plans
// change the partial counts).
static size_t workspace_all(const gpspca_matrix* A, int form, int m, int max_iter, int ncu,
                            int path) {
    size_t mx = 0;
    for (const Tune& t : tune_candidates(A, m, path)) {
        Plan pl;
        make_plan(A, form, m, max_iter, ncu, &pl, path, 0, &t);
        mx = std::max(mx, pl.total);
    }
    {
        Plan pe;  // the plan the environment or the autotuner's table selects
        make_plan(A, form, m, max_iter, ncu, &pe, path, 0);
        mx = std::max(mx, pe.total);
    }
    if (A->dtype == GPSPCA_F32) {
        Plan pr;  // frozen-support passes (refinement) on the same matrix
        make_plan(A, form, m, max_iter, ncu, &pr, path, 1);
        mx = std::max(mx, pr.total);
    }
    return mx;
}

struct Ptrs {
    float* xpart;
    Ctrl* ctrl;
    double* trace;
    float* x[2];
    float* S;
    uint8_t* act;
    float* gpart;
    int* touched;
    double* fpart;
    int* nnzpart;
    double* l1;
    double* g64;
    double* gram;
    double* coef;
    double* norms;
    double* cand_v;
    int64_t* cand_i;
    int64_t* idx;
    double* fin;
    double* invn;
    double* fcomp;
    PathState* pstate;
    int* list;
    int* nlist;
    float* xil[2];
    double* fsum;
};

static Ptrs carve(const Plan& pl, void* ws) {
    char* b = static_cast<char*>(ws);
    Ptrs P;
    P.ctrl = reinterpret_cast<Ctrl*>(b + pl.o_ctrl);
    P.trace = reinterpret_cast<double*>(b + pl.o_trace);
    P.x[0] = reinterpret_cast<float*>(b + pl.o_x0);
    P.x[1] = reinterpret_cast<float*>(b + pl.o_x1);
    P.S = reinterpret_cast<float*>(b + pl.o_s);
    P.act = reinterpret_cast<uint8_t*>(b + pl.o_act);
    P.gpart = reinterpret_cast<float*>(b + pl.o_gpart);
    P.touched = reinterpret_cast<int*>(b + pl.o_touched);
    P.fpart = reinterpret_cast<double*>(b + pl.o_fpart);
    P.nnzpart = reinterpret_cast<int*>(b + pl.o_nnzpart);
    P.l1 = reinterpret_cast<double*>(b + pl.o_l1);
    P.g64 = reinterpret_cast<double*>(b + pl.o_g64);
    P.gram = reinterpret_cast<double*>(b + pl.o_gram);
    P.coef = reinterpret_cast<double*>(b + pl.o_coef);
    P.norms = reinterpret_cast<double*>(b + pl.o_norms);
    P.cand_v = reinterpret_cast<double*>(b + pl.o_cand_v);
    P.cand_i = reinterpret_cast<int64_t*>(b + pl.o_cand_i);
    P.idx = reinterpret_cast<int64_t*>(b + pl.o_idx);
    P.fin = reinterpret_cast<double*>(b + pl.o_fin);
    P.invn = reinterpret_cast<double*>(b + pl.o_invn);
    P.fcomp = reinterpret_cast<double*>(b + pl.o_fcomp);
    P.pstate = reinterpret_cast<PathState*>(b + pl.o_pstate);
    P.list = reinterpret_cast<int*>(b + pl.o_list);
    P.nlist = P.list + pl.n;
    P.xil[0] = reinterpret_cast<float*>(b + pl.o_xil0);
    P.xil[1] = reinterpret_cast<float*>(b + pl.o_xil1);
    P.fsum = reinterpret_cast<double*>(b + pl.o_fsum);
    P.xpart = reinterpret_cast<float*>(b + pl.o_xpart);
    return P;
}

static PassParams make_params(const gpspca_matrix* A, const Plan& pl, double gamma,
                              const double* mu, const double* gammas = nullptr) {
    PassParams pp;
    std::memset(&pp, 0, sizeof(pp));
    if (A->dtype == GPSPCA_BF16) pp.Abf = static_cast<const uint16_t*>(A->data);
    else if (A->dtype == GPSPCA_F8E4M3) pp.Af8 = static_cast<const uint8_t*>(A->data);
    else pp.A = static_cast<const float*>(A->data);
    pp.scale = A->col_scale;
    pp.lda = A->lda;
    pp.n = A->n;
    pp.p = (int)A->p;
    pp.ldx = pl.ldx;
    pp.m = pl.m;
    pp.l0 = pl.l0;
    pp.gamma = gamma;
    const bool block = pl.form >= GPSPCA_BL1;
    for (int j = 0; j < kMaxM; ++j) {
        const double v = (block && mu && j < pl.m) ? mu[j] : 1.0;
        pp.mu[j] = v;
        pp.muf[j] = (float)v;
        pp.gam[j] = (gammas && j < pl.m) ? gammas[j] : gamma;
    }
    return pp;
}

// ------------------------------------------------------------------ profiling
struct Prof {
    std::mutex mu;
    bool on = false;
    int every = 1;   // time one launch in `every`
    double total_ms = 0.0;
    int64_t launches = 0;
    std::string name;
};
static Prof g_prof;

thread_local KernelEvents g_kev;

// Event pairs of the timed launches, kept for the thread's later solves: a
// pair is created once, not per solve, so that the first pass of a solve does
// not wait for the host to create its events.
struct EventPool {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    ~EventPool() {
        for (auto& e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};
static thread_local EventPool t_events;

struct TimedLaunches {
    size_t used = 0;    // pairs of t_events taken by this solve
    bool on = false;
    int every = 1;
    int64_t seen = 0;
    bool cur = false;   // the current launch is timed
    ~TimedLaunches() { g_kev = KernelEvents{}; }
    // The correlation launch between begin() and end() records the pair at
    // its own start and end (GPSPCA_LAUNCH_TIMED); an event pair recorded
    // around it measured 9 us more than the kernel's own duration (718.8
    // against 709.8 us on 10000 x 100000, m = 8).
    hipError_t begin(hipStream_t st) {
        (void)st;
        cur = on && (seen++ % every) == 0;
        if (!cur) return hipSuccess;
        if (used == t_events.ev.size()) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreateWithFlags(&a, hipEventDisableSystemFence);
            if (e != hipSuccess) return e;
            e = hipEventCreateWithFlags(&b, hipEventDisableSystemFence);
            if (e != hipSuccess) {
                (void)hipEventDestroy(a);
                return e;
            }
            t_events.ev.emplace_back(a, b);
        }
        const auto& pr = t_events.ev[used++];
        g_kev.start = pr.first;
        g_kev.stop = pr.second;
        return hipSuccess;
    }
    hipError_t end(hipStream_t st) {
        (void)st;
        g_kev = KernelEvents{};
        return hipSuccess;
    }
    void collect(const char* name) {
        if (!on) return;
        double tot = 0.0;
        int64_t n = 0;
        for (size_t i = 0; i < used; ++i) {
            const auto& e = t_events.ev[i];
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
                tot += ms;
                ++n;
            }
        }
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.total_ms += tot;
        g_prof.launches += n;
        g_prof.name = name;
    }
};

// ----------------------------------------------------------------- driver
static int enqueue_pass(const Plan& pl, const PassParams& pp, const Ptrs& P, int k,
                        hipStream_t st, TimedLaunches& tl) {
    const float* Xk = P.x[k & 1];
    float* Xn = P.x[(k + 1) & 1];
    const int* touched = pl.fused_m1 ? nullptr : P.touched;
    GPSPCA_HIP(tl.begin(st));
    if (pl.fused_m1) {
        GPSPCA_HIP(launch_pass_m1(pl, pp, Xk, P.S, P.gpart, P.fpart, P.nnzpart, P.ctrl, st));
        GPSPCA_HIP(tl.end(st));
    } else {
        if (pl.use_vx)
            GPSPCA_HIP(launch_corr_vx(pl, pp, Xk, P.S, P.act, P.fpart, P.nnzpart, P.ctrl, st));
        else if (pl.use_mv)
            GPSPCA_HIP(launch_corr_mv(pl, pp, Xk, P.S, P.act, P.fpart, P.nnzpart, P.ctrl, st));
        else if (pl.use_qw)
            GPSPCA_HIP(launch_corr_qw(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                      P.ctrl, st));
        else if (pl.use_q)
            GPSPCA_HIP(launch_corr_q(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                     P.ctrl, st));
        else if (pl.use_x3)
            GPSPCA_HIP(launch_corr_x3(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                      P.ctrl, st));
        else if (pl.use_rd)
            GPSPCA_HIP(launch_corr_rd(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                      P.ctrl, st));
        else if (pl.use_wg)
            GPSPCA_HIP(launch_corr_wg(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                      P.ctrl, st));
        else if (pl.use_mfma)
            GPSPCA_HIP(launch_corr_mfma(pl, pp, Xk, P.xil[k & 1], P.S, P.act, P.fpart, P.nnzpart,
                                        P.xpart, P.ctrl, st));
        else
            GPSPCA_HIP(launch_corr(pl, pp, Xk, P.S, P.act, P.fpart, P.nnzpart, P.ctrl, st));
        GPSPCA_HIP(tl.end(st));
        GPSPCA_HIP(launch_backproj(pl, pp, P.S, P.act, P.gpart, P.touched, P.ctrl, st));
    }
    const int with_x = pl.path ? 2 : (pl.m > 1 ? 1 : 0);
    if (pl.fused_m1) {
        GPSPCA_HIP(launch_reduce_m1(pl, P.gpart, P.g64, P.gram, P.ctrl, st));
    } else if (pl.fused_gram) {
        GPSPCA_HIP(launch_reduce_gram(pl, P.gpart, touched, Xk, with_x, P.g64, P.gram, P.ctrl, st));
    } else {
        GPSPCA_HIP(launch_reduce_partials(pl, P.gpart, touched, P.l1, P.ctrl, st));
        GPSPCA_HIP(launch_gram(pl, P.l1, pl.red_split, Xk, with_x, P.g64, P.gram, P.ctrl, st));
    }
    // single-unit passes whose x needs no interleaved copy: the stop kernel
    // writes x_{k+1} = g / ||g|| itself (one launch less per pass)
    const bool x_in_stop = !pl.path && pl.m == 1 && pl.defl_k == 0 && !(pl.use_mfma || pl.use_q);
    if (pl.path) {
        GPSPCA_HIP(launch_stop_path(pl, P.fpart, P.nnzpart, P.gram, P.trace, P.coef, P.fcomp,
                                    P.pstate, P.ctrl, st));
    } else {
        GPSPCA_HIP(launch_stop(pl, P.fpart, P.nnzpart, P.gram, P.trace, P.coef, P.fcomp,
                               P.coef + 5 * (size_t)pl.m * pl.m, P.g64, x_in_stop ? Xn : nullptr,
                               P.fsum, P.ctrl, st));
    }
    if (x_in_stop) return GPSPCA_OK;
    if (pl.defl_k > 0) {
        // deflated component (m = 1): x_{k+1} = P g / ||P g|| straight from the
        // FP64 g, which the normalization of the plain retraction would only scale
        GPSPCA_HIP(launch_deflate((int)pl.p, pl.defl_k, pl.defl_q, P.g64, Xn, P.g64,
                                  P.ctrl, st));
        if (pl.use_mfma || pl.use_q) GPSPCA_HIP(launch_x_interleave(pl, Xn, P.xil[(k + 1) & 1], st));
    } else {
        GPSPCA_HIP(launch_apply(pl, P.g64, Xk, P.coef, Xn,
                                (pl.use_mfma || pl.use_q) ? P.xil[(k + 1) & 1] : nullptr, P.ctrl,
                                st));
    }
    return GPSPCA_OK;
}

struct Pinned {
    Ctrl* snap = nullptr;
    void* stage = nullptr;     // outputs read back with the control block
    size_t stage_cap = 0;
    ~Pinned() {
        if (snap) (void)hipHostFree(snap);
        if (stage) (void)hipHostFree(stage);
    }
};
static thread_local Pinned t_pinned;

// Pinned host memory of at least `bytes` (64 KB at least, kept for the thread's
// later calls, so that a solve allocates it only when it needs more).
static int pinned_stage(size_t bytes, void** out) {
    if (t_pinned.stage_cap < bytes) {
        size_t cap = (size_t)64 << 10;
        while (cap < bytes) cap *= 2;
        if (t_pinned.stage) GPSPCA_HIP(hipHostFree(t_pinned.stage));
        t_pinned.stage = nullptr;
        t_pinned.stage_cap = 0;
        void* p = nullptr;
        GPSPCA_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
        t_pinned.stage = p;
        t_pinned.stage_cap = cap;
    }
    *out = t_pinned.stage;
    return GPSPCA_OK;
}

static int pinned_ctrl(Ctrl** out) {
    if (!t_pinned.snap) {
        void* p = nullptr;
        GPSPCA_HIP(hipHostMalloc(&p, sizeof(Ctrl), hipHostMallocDefault));
        t_pinned.snap = static_cast<Ctrl*>(p);
    }
    *out = t_pinned.snap;
    return GPSPCA_OK;
}


// Two consecutive passes (even then odd k: the X buffers alternate) captured
// as one HIP graph, replayed for every pair of passes of a solve.  Capture runs
// on a private stream (the legacy default stream cannot capture); the graph is
// launched on the caller's stream.  Every pass kernel reads its pass index and
// stop flag from the device control block, so a replay is the same work as
// enqueuing the pair again.
struct PassGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    ~PassGraph() {
        if (ex) (void)hipGraphExecDestroy(ex);
        if (g) (void)hipGraphDestroy(g);
    }
};

// Graphs are used for small matrices only (at most 256 MB of A), where launch
// latency is a large share of a pass; GPSPCA_GRAPH=0 / 1 forces them off / on.
// On large matrices the replayed pair measured slower than the same passes
// enqueued one by one (10000 x 100000, m = 8: 844 against 760 us per pass;
// 5000 x 50000, m = 1: 173 against 167 us).
static bool graphs_enabled(const Plan& pl) {
    const char* e = std::getenv("GPSPCA_GRAPH");
    if (e && e[0] == '0') return false;
    if (e && e[0] == '1') return true;
    const double elem = pl.dtype == GPSPCA_BF16 ? 2.0 : pl.dtype == GPSPCA_F8E4M3 ? 1.0 : 4.0;
    return (double)pl.p * (double)pl.n * elem <= 256.0 * (1 << 20);
}

static int capture_pair(const Plan& pl, const PassParams& pp, const Ptrs& P, PassGraph* pg) {
    static thread_local hipStream_t cap = nullptr;
    if (!cap) GPSPCA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    GPSPCA_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    TimedLaunches none;
    int rc = enqueue_pass(pl, pp, P, 0, cap, none);
    if (!rc) rc = enqueue_pass(pl, pp, P, 1, cap, none);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(GPSPCA_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    pg->g = g;
    GPSPCA_HIP(hipGraphInstantiate(&pg->ex, g, nullptr, nullptr, 0));
    return GPSPCA_OK;
}

// Enqueue passes in growing chunks; the stopping rule runs on the device and
// the host reads the control block once per chunk (with tol = 0 every pass is
// enqueued at once).  Pairs of passes go through a captured graph when the
// solve is long enough to repay the capture (and kernel timing is off).
// Returns the final control block in *fin.
// tail: work enqueued after the last pass and before the control block is read
// back (the solve's outputs), so that the host waits once.
// noalloc: no graph (instantiation allocates), no launch timing (events), and
// the control block is read into the caller's stack instead of pinned memory.
static int run_passes(const Plan& pl, const PassParams& pp, const Ptrs& P, int max_iter,
                      double tol, hipStream_t st, Ctrl* fin, bool noalloc = false,
                      const std::function<int()>* tail = nullptr) {
    TimedLaunches tl;
    if (!noalloc) {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        tl.on = g_prof.on;
        tl.every = g_prof.every;
    }
    Ctrl stack_snap;
    Ctrl* snap = &stack_snap;
    int rc = noalloc ? GPSPCA_OK : pinned_ctrl(&snap);
    if (rc) return rc;
    PassGraph pg;
    const bool use_graph = !noalloc && !tl.on && max_iter >= 8 && graphs_enabled(pl);
    if (use_graph) {
        rc = capture_pair(pl, pp, P, &pg);
        if (rc) return rc;
    }
    int kk = 0;
    int chunk = (tol == 0.0) ? max_iter : (use_graph ? 2 : 1);
    while (kk < max_iter) {
        const int c = std::min(chunk, max_iter - kk);
        int i = 0;
        if (use_graph)
            for (; i + 1 < c; i += 2) GPSPCA_HIP(hipGraphLaunch(pg.ex, st));
        for (; i < c; ++i) {
            rc = enqueue_pass(pl, pp, P, kk + i, st, tl);
            if (rc) return rc;
        }
        kk += c;
        if (kk >= max_iter) break;
        GPSPCA_HIP(hipMemcpyAsync(snap, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        GPSPCA_HIP(hipStreamSynchronize(st));
        if (snap->done) break;
        chunk = std::min(chunk * 2, 32);
    }
    if (tail) {
        rc = (*tail)();
        if (rc) return rc;
    }
    GPSPCA_HIP(hipMemcpyAsync(snap, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    GPSPCA_HIP(hipStreamSynchronize(st));
    tl.collect(pl.fused_m1 ? "k_pass_m1"
                           : pl.use_vx ? "k_corr_vx"
                           : pl.use_mv ? "k_corr_mv"
                           : pl.use_qw ? "k_corr_qw"
                           : pl.use_q ? "k_corr_q"
                           : pl.use_x3 ? "k_corr_x3"
                           : pl.use_rd ? "k_corr_rd"
                           : pl.use_wg ? "k_corr_wg"
                           : pl.use_mfma ? "k_corr_mfma" : "k_corr");
    *fin = *snap;
    return GPSPCA_OK;
}

static const char* status_text(int s) {
    switch (s) {
        case GPSPCA_EINVAL: return "rank-deficient or zero starting point";
        case GPSPCA_ENONFINITE: return "objective or ascent direction became non-finite";
        default: return "device error";
    }
}


// One driver for every iteration entry point.
//  path = 0: one problem (form, m, gamma, mu); path = 1: m independent
//  single-unit problems with their own gammas[j] (a gamma path).
//  mask != nullptr: frozen-support passes (X0 required): only the columns with
//  a support bit are read and s_ij = 0 wherever bit (i, j) is clear.
//  norms_in != nullptr: device column norms of A for the default start (the
//  server caches them with a resident matrix).
//  multistart (path, no X0): problem j starts at the normalized column of the
//  j-th largest norm instead of all at the largest.
int solve_core(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
               const double* gammas, int path, const uint32_t* mask, const float* X0,
               double tol, int max_iter, void* workspace, size_t ws_bytes, hipStream_t st,
               float* X, float* Z, uint32_t* support, double* obj_trace, int* n_iter,
               int* status_out, const double* norms_in, int multistart, const double* defl_q,
               int defl_k, int exact, int noalloc) {
    int ncu = 0;
    int rc = device_cus(&ncu);
    if (rc) return rc;
    const int pform = path ? (form == GPSPCA_SL0 ? GPSPCA_BL0 : GPSPCA_BL1) : form;
    Plan pl;
    make_plan(A, pform, m, max_iter, ncu, &pl, path, mask ? 1 : 0);
    if (ws_bytes < pl.total) return fail(GPSPCA_ENOMEM, "workspace too small");
    pl.defl_q = defl_q;
    pl.defl_k = defl_q ? defl_k : 0;
    pl.exact = (exact && !path) ? 1 : 0;
    const Ptrs P = carve(pl, workspace);
    PassParams pp = make_params(A, pl, gamma, mu, gammas);
    pp.nact = &P.ctrl->nact;
    const int64_t words = cdiv(A->n, 32);

    // one launch resets the control block, clears the X buffers (their padding
    // rows and components stay zero), their interleaved copies (written by the
    // start's retraction and by every pass's), the path state and, for
    // frozen-support passes, S and the activity flags, and loads X0
    const bool il = pl.use_mfma || pl.use_q;
    StartZero z{};
    auto zero = [&](void* ptr, size_t bytes) {
        z.ptr[z.n] = static_cast<uint32_t*>(ptr);
        z.words[z.n] = bytes / 4;
        ++z.n;
    };
    zero(P.x[0], sizeof(float) * pl.ldx * pl.mpad);
    zero(P.x[1], sizeof(float) * pl.ldx * pl.mpad);
    if (il) {
        zero(P.xil[0], pl.xil_bytes);
        zero(P.xil[1], pl.xil_bytes);
    }
    if (path) zero(P.pstate, sizeof(PathState) * m);
    if (mask) {
        zero(P.S, sizeof(float) * (size_t)A->n * m);
        zero(P.act, align_up((size_t)A->n, 4));
    }
    GPSPCA_HIP(launch_start(P.ctrl, max_iter, tol, z, m, (int)A->p, X0, (int)A->p, P.g64, st));
    if (mask) {
        GPSPCA_HIP(launch_mask_list(mask, words, m, A->n, P.list, P.nlist, st));
        pp.list = P.list;
        pp.nlist = P.nlist;
        pp.mask = mask;
        pp.mask_words = words;
    }

    // start: project X0 (or the default start) onto the feasible set
    // the retraction that ends each start writes X_0 and, for the matrix-core
    // kernels, its interleaved copy (except the broadcast start, copied after)
    float* xil0 = il ? P.xil[0] : nullptr;
    if (X0) {
        if (path) {
            // every column normalized on its own
            GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 2, P.g64, P.gram, P.ctrl, st));
            GPSPCA_HIP(launch_project_diag(pl, P.gram, P.coef, P.ctrl, st));
        } else {
            GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 0, P.g64, P.gram, P.ctrl, st));
            GPSPCA_HIP(launch_project(pl, P.gram, P.coef, P.ctrl, st));
        }
        GPSPCA_HIP(launch_apply(pl, P.g64, P.x[1], P.coef, P.x[0], xil0, P.ctrl, st));
    } else if (path && multistart) {
        // problem j starts at the column of the j-th largest norm (ties to the
        // lower index), normalized on its own
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2LL * ncu, cdiv(A->n, 16)));
        if (!norms_in) GPSPCA_HIP(launch_colnorm(pp, A->dtype, P.norms, grid, st));
        GPSPCA_HIP(launch_topm(pl, norms_in ? norms_in : P.norms, P.cand_v, P.cand_i, P.idx, st));
        GPSPCA_HIP(launch_gather(pl, pp, P.idx, P.g64, st));
        GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 2, P.g64, P.gram, P.ctrl, st));
        GPSPCA_HIP(launch_project_diag(pl, P.gram, P.coef, P.ctrl, st));
        GPSPCA_HIP(launch_apply(pl, P.g64, P.x[1], P.coef, P.x[0], xil0, P.ctrl, st));
    } else if (path) {
        // all columns start at the normalized column of largest norm
        Plan p1;
        make_plan(A, GPSPCA_SL1, 1, 1, ncu, &p1);
        p1.ldx = pl.ldx;
        p1.gram_grid = pl.gram_grid;
        p1.gram_rows = pl.gram_rows;
        p1.topm_grid = pl.topm_grid;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2LL * ncu, cdiv(A->n, 16)));
        if (!norms_in) GPSPCA_HIP(launch_colnorm(pp, A->dtype, P.norms, grid, st));
        GPSPCA_HIP(launch_topm(p1, norms_in ? norms_in : P.norms, P.cand_v, P.cand_i, P.idx, st));
        PassParams pp1 = pp;
        pp1.m = 1;
        GPSPCA_HIP(launch_gather(p1, pp1, P.idx, P.g64, st));
        GPSPCA_HIP(launch_gram(p1, nullptr, 0, nullptr, 0, P.g64, P.gram, P.ctrl, st));
        GPSPCA_HIP(launch_project(p1, P.gram, P.coef, P.ctrl, st));
        GPSPCA_HIP(launch_apply(p1, P.g64, P.x[1], P.coef, P.x[0], nullptr, P.ctrl, st));
        GPSPCA_HIP(launch_bcast_col0(pl, P.x[0], st));
        if (il) GPSPCA_HIP(launch_x_interleave(pl, P.x[0], P.xil[0], st));
    } else {
        // the m columns of largest norm (ties to the lower index)
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2LL * ncu, cdiv(A->n, 16)));
        if (!norms_in) GPSPCA_HIP(launch_colnorm(pp, A->dtype, P.norms, grid, st));
        GPSPCA_HIP(launch_topm(pl, norms_in ? norms_in : P.norms, P.cand_v, P.cand_i, P.idx, st));
        GPSPCA_HIP(launch_gather(pl, pp, P.idx, P.g64, st));
        GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 0, P.g64, P.gram, P.ctrl, st));
        GPSPCA_HIP(launch_project(pl, P.gram, P.coef, P.ctrl, st));
        GPSPCA_HIP(launch_apply(pl, P.g64, P.x[1], P.coef, P.x[0], xil0, P.ctrl, st));
    }

    // outputs, enqueued behind the passes: the copy of X takes the last
    // iterate by the pass count on the device, and the trace and path state
    // come back into pinned memory with the control block (one wait in all)
    const size_t trace_n = obj_trace ? (path ? (size_t)m * max_iter : (size_t)max_iter) : 0;
    const size_t stage_bytes = sizeof(double) * trace_n + (path ? sizeof(PathState) * m : 0);
    void* stage = nullptr;
    if (!noalloc && stage_bytes) {
        rc = pinned_stage(stage_bytes, &stage);
        if (rc) return rc;
    }
    char* const stage_ps = static_cast<char*>(stage) + sizeof(double) * trace_n;
    const std::function<int()> outputs = [&]() -> int {
        GPSPCA_HIP(launch_copy_x_last(pl, P.x[0], P.x[1], P.ctrl, X, st));
        GPSPCA_HIP(launch_finalize(pl, P.S, P.fin, P.invn, Z, support, st));
        if (stage && trace_n)
            GPSPCA_HIP(hipMemcpyAsync(stage, P.trace, sizeof(double) * trace_n,
                                      hipMemcpyDeviceToHost, st));
        if (stage && path)
            GPSPCA_HIP(hipMemcpyAsync(stage_ps, P.pstate, sizeof(PathState) * m,
                                      hipMemcpyDeviceToHost, st));
        return GPSPCA_OK;
    };
    Ctrl fin;
    rc = run_passes(pl, pp, P, max_iter, tol, st, &fin, noalloc != 0, &outputs);
    if (rc) return rc;
    if (fin.status < 0) return fail(fin.status, status_text(fin.status));
    if (fin.n_iter < 1) return fail(GPSPCA_EDEVICE, "solve ended without a pass");

    std::vector<PathState> ps(path ? m : 0);
    const size_t cnt = path ? (size_t)m * max_iter : (size_t)fin.n_iter;
    if (stage) {
        if (obj_trace) std::memcpy(obj_trace, stage, sizeof(double) * cnt);
        if (path) std::memcpy(ps.data(), stage_ps, sizeof(PathState) * m);
    } else if (path || obj_trace) {
        if (path)
            GPSPCA_HIP(hipMemcpyAsync(ps.data(), P.pstate, sizeof(PathState) * m,
                                      hipMemcpyDeviceToHost, st));
        if (obj_trace)
            GPSPCA_HIP(hipMemcpyAsync(obj_trace, P.trace, sizeof(double) * cnt,
                                      hipMemcpyDeviceToHost, st));
        GPSPCA_HIP(hipStreamSynchronize(st));
    }
    if (!path) {
        if (n_iter) *n_iter = fin.n_iter;
        if (fin.status != GPSPCA_OK)
            g_err = fin.status == GPSPCA_MAXITER ? "stopped at max_iter" : "degenerate components";
        return fin.status;
    }
    int worst = GPSPCA_OK;
    for (int j = 0; j < m; ++j) {
        if (n_iter) n_iter[j] = ps[j].n_iter;
        if (status_out) status_out[j] = ps[j].status;
        if (ps[j].status < 0) worst = ps[j].status;
        else if (worst >= 0 && ps[j].status > worst) worst = ps[j].status;
    }
    if (worst < 0) return fail(worst, status_text(worst));
    return worst;
}

static int check_run(double tol, int max_iter, const float* X, const void* workspace) {
    if (!std::isfinite(tol) || tol < 0.0) return fail(GPSPCA_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 1) return fail(GPSPCA_EINVAL, "max_iter must be >= 1");
    if (!X) return fail(GPSPCA_EINVAL, "X is NULL");
    if (!workspace) return fail(GPSPCA_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(GPSPCA_EINVAL, "workspace must be 256-byte aligned");
    return GPSPCA_OK;
}

static int check_path(const gpspca_matrix* A, int form, int K, const double* gammas) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (form != GPSPCA_SL1 && form != GPSPCA_SL0)
        return fail(GPSPCA_EINVAL, "a gamma path takes a single-unit formulation");
    if (K < 1 || K > kMaxM) return fail(GPSPCA_EINVAL, "need 1 <= K <= GPSPCA_MAX_M");
    if (!gammas) return fail(GPSPCA_EINVAL, "gammas is NULL");
    for (int j = 0; j < K; ++j)
        if (!std::isfinite(gammas[j]) || gammas[j] < 0.0)
            return fail(GPSPCA_EINVAL, "gammas must be finite and >= 0");
    return GPSPCA_OK;
}

// ------------------------------------------------------- allocation-free solve
// Scratch of gpspca_solve_noalloc, in place of the caller's workspace: one copy
// per GPU (each device holds its own at its own address until the process
// ends).  On the host the array's name is only a stand-in for the device
// symbol; host code uses the device address that hipGetSymbolAddress returns,
// resolved once per device with that device current, and never the name.
static __device__ __align__(256) unsigned char scratch[GPSPCA_NOALLOC_SCRATCH_BYTES];

static int scratch_address(void** out) {
    static std::mutex mu;
    static void* addr[64] = {nullptr};
    int dev = 0;
    GPSPCA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(GPSPCA_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* ptr = nullptr;
        GPSPCA_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
            return fail(GPSPCA_EDEVICE, "scratch symbol has no aligned device address");
        addr[dev] = ptr;
    }
    *out = addr[dev];
    return GPSPCA_OK;
}

}  // namespace gpspca

using namespace gpspca;

extern "C" {

const char* gpspca_last_error(void) { return g_err.c_str(); }

const char* gpspca_version(void) { return "gpspca-gfx950 0.1"; }

size_t gpspca_workspace_bytes(const gpspca_matrix* A, int form, int m, int max_iter) {
    if (form == GPSPCA_BL1X) form = GPSPCA_BL1;  // the same passes
    if (check_problem(A, form, m, 0.0, nullptr) != GPSPCA_OK) return 0;
    if (max_iter < 1) {
        fail(GPSPCA_EINVAL, "max_iter must be >= 1");
        return 0;
    }
    int ncu = 0;
    if (device_cus(&ncu) != GPSPCA_OK) return 0;
    return workspace_all(A, form, m, max_iter, ncu, 0);
}

int gpspca_solve(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                 const float* X0, double tol, int max_iter, void* workspace, size_t ws_bytes,
                 void* stream, float* X, float* Z, uint32_t* support, double* obj_trace,
                 int* n_iter) {
    // BL1X runs BL1's passes with the original form's objective and retraction
    const int exact = form == GPSPCA_BL1X ? 1 : 0;
    if (exact) form = GPSPCA_BL1;
    int rc = check_problem(A, form, m, gamma, mu);
    if (rc) return rc;
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    if (!X0 && m > A->n) return fail(GPSPCA_EINVAL, "default start needs m <= n");
    return solve_core(A, form, m, gamma, mu, nullptr, 0, nullptr, X0, tol, max_iter, workspace,
                      ws_bytes, static_cast<hipStream_t>(stream), X, Z, support, obj_trace,
                      n_iter, nullptr, nullptr, 0, nullptr, 0, exact);
}

int gpspca_solve_noalloc(const gpspca_matrix* A, int form, int m, double gamma,
                         const double* mu, const float* X0, double tol, int max_iter,
                         void* stream, float* X, float* Z, uint32_t* support,
                         double* obj_trace, int* n_iter) {
    const int exact = form == GPSPCA_BL1X ? 1 : 0;
    if (exact) form = GPSPCA_BL1;
    int rc = check_problem(A, form, m, gamma, mu);
    if (rc) return rc;
    if (!std::isfinite(tol) || tol < 0.0) return fail(GPSPCA_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 1) return fail(GPSPCA_EINVAL, "max_iter must be >= 1");
    if (!X) return fail(GPSPCA_EINVAL, "X is NULL");
    if (!X0 && m > A->n) return fail(GPSPCA_EINVAL, "default start needs m <= n");
    int ncu = 0;
    rc = device_cus(&ncu);
    if (rc) return rc;
    Plan pl;  // the plan solve_core will make
    make_plan(A, form, m, max_iter, ncu, &pl);
    if (pl.total > GPSPCA_NOALLOC_SCRATCH_BYTES)
        return fail(GPSPCA_ENOMEM, "problem needs " + std::to_string(pl.total) +
                                       " bytes of scratch, more than GPSPCA_NOALLOC_SCRATCH_BYTES (" +
                                       std::to_string((size_t)GPSPCA_NOALLOC_SCRATCH_BYTES) + ")");
    void* ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    return solve_core(A, form, m, gamma, mu, nullptr, 0, nullptr, X0, tol, max_iter, ws,
                      GPSPCA_NOALLOC_SCRATCH_BYTES, static_cast<hipStream_t>(stream), X, Z,
                      support, obj_trace, n_iter, nullptr, nullptr, 0, nullptr, 0, exact, 1);
}

int gpspca_refine(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                  const uint32_t* support_in, const float* X0, double tol, int max_iter,
                  void* workspace, size_t ws_bytes, void* stream, float* X, float* Z,
                  uint32_t* support, double* obj_trace, int* n_iter) {
    int rc = check_problem(A, form, m, gamma, mu);
    if (rc) return rc;
    if (A->dtype != GPSPCA_F32) return fail(GPSPCA_EDTYPE, "refinement runs on FP32 storage");
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    if (!support_in) return fail(GPSPCA_EINVAL, "support is NULL");
    if (!X0) return fail(GPSPCA_EINVAL, "refinement needs X0");
    return solve_core(A, form, m, gamma, mu, nullptr, 0, support_in, X0, tol, max_iter,
                      workspace, ws_bytes, static_cast<hipStream_t>(stream), X, Z, support,
                      obj_trace, n_iter, nullptr, nullptr);
}

int gpspca_step(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                const float* Xin, void* workspace, size_t ws_bytes, void* stream, float* S,
                double* G, double* f, int64_t* nnz) {
    int rc = check_problem(A, form, m, gamma, mu);
    if (rc) return rc;
    if (!Xin) return fail(GPSPCA_EINVAL, "X is NULL");
    if (!workspace) return fail(GPSPCA_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(GPSPCA_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int ncu = 0;
    rc = device_cus(&ncu);
    if (rc) return rc;
    Plan pl;
    make_plan(A, form, m, 1, ncu, &pl);
    if (ws_bytes < pl.total) return fail(GPSPCA_ENOMEM, "workspace too small");
    const Ptrs P = carve(pl, workspace);
    PassParams pp = make_params(A, pl, gamma, mu);
    pp.nact = &P.ctrl->nact;
    GPSPCA_HIP(launch_ctrl_reset(P.ctrl, 1, 0.0, st));
    GPSPCA_HIP(launch_fill_zero(P.x[0], sizeof(float) * pl.ldx * pl.mpad, st));
    GPSPCA_HIP(hipMemcpy2DAsync(P.x[0], sizeof(float) * pl.ldx, Xin, sizeof(float) * A->p,
                                sizeof(float) * A->p, m, hipMemcpyDeviceToDevice, st));
    if (pl.use_mfma || pl.use_q) GPSPCA_HIP(launch_x_interleave(pl, P.x[0], P.xil[0], st));
    TimedLaunches tl;
    rc = enqueue_pass(pl, pp, P, 0, st, tl);
    if (rc) return rc;
    if (S) GPSPCA_HIP(launch_finalize(pl, P.S, P.fin, nullptr, S, nullptr, st));
    if (G)
        GPSPCA_HIP(hipMemcpyAsync(G, P.g64, sizeof(double) * m * A->p, hipMemcpyDeviceToDevice, st));
    std::vector<double> host(2 * (size_t)m);
    GPSPCA_HIP(hipMemcpyAsync(host.data(), P.fcomp, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st));
    Ctrl* snap = nullptr;
    rc = pinned_ctrl(&snap);
    if (rc) return rc;
    GPSPCA_HIP(hipMemcpyAsync(snap, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    GPSPCA_HIP(hipStreamSynchronize(st));
    if (snap->status == GPSPCA_ENONFINITE) return fail(GPSPCA_ENONFINITE, status_text(GPSPCA_ENONFINITE));
    for (int j = 0; j < m; ++j) {
        if (f) f[j] = host[j];
        if (nnz) std::memcpy(&nnz[j], &host[m + j], sizeof(int64_t));
    }
    return GPSPCA_OK;
}

size_t gpspca_path_workspace_bytes(const gpspca_matrix* A, int K, int max_iter) {
    if (check_matrix(A) != GPSPCA_OK) return 0;
    if (K < 1 || K > kMaxM) {
        fail(GPSPCA_EINVAL, "need 1 <= K <= GPSPCA_MAX_M");
        return 0;
    }
    if (max_iter < 1) {
        fail(GPSPCA_EINVAL, "max_iter must be >= 1");
        return 0;
    }
    int ncu = 0;
    if (device_cus(&ncu) != GPSPCA_OK) return 0;
    return workspace_all(A, GPSPCA_BL1, K, max_iter, ncu, 1);
}

int gpspca_solve_path(const gpspca_matrix* A, int form, int K, const double* gammas,
                      const float* X0, double tol, int max_iter, void* workspace,
                      size_t ws_bytes, void* stream, float* X, float* Z, uint32_t* support,
                      double* obj_trace, int* n_iter, int* status) {
    int rc = check_path(A, form, K, gammas);
    if (rc) return rc;
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    return solve_core(A, form, K, 0.0, nullptr, gammas, 1, nullptr, X0, tol, max_iter, workspace,
                      ws_bytes, static_cast<hipStream_t>(stream), X, Z, support, obj_trace,
                      n_iter, status, nullptr, 0);
}

int gpspca_solve_multistart(const gpspca_matrix* A, int form, int m, double gamma, double tol,
                            int max_iter, void* workspace, size_t ws_bytes, void* stream,
                            float* X, float* Z, uint32_t* support, double* obj_trace,
                            int* n_iter, int* status) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (m > A->n) return fail(GPSPCA_EINVAL, "multi-start needs m <= n");
    std::vector<double> gammas((size_t)std::max(0, std::min(m, kMaxM)), gamma);
    rc = check_path(A, form, m, gammas.data());
    if (rc) return rc;
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    return solve_core(A, form, m, 0.0, nullptr, gammas.data(), 1, nullptr, nullptr, tol,
                      max_iter, workspace, ws_bytes, static_cast<hipStream_t>(stream), X, Z,
                      support, obj_trace, n_iter, status, nullptr, 1);
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// The single-unit solve's share of a deflation workspace (either form).
static size_t deflated_core(const gpspca_matrix* A, int max_iter, int ncu) {
    return al256(std::max(workspace_all(A, GPSPCA_SL1, 1, max_iter, ncu, 0),
                          workspace_all(A, GPSPCA_SL0, 1, max_iter, ncu, 0)));
}

size_t gpspca_deflated_workspace_bytes(const gpspca_matrix* A, int m, int max_iter) {
    if (check_problem(A, GPSPCA_SL1, 1, 0.0, nullptr) != GPSPCA_OK) return 0;
    if (m < 1 || m > kMaxM || m > A->p || m > A->n) {
        fail(GPSPCA_EINVAL, "need 1 <= m <= min(p, n, GPSPCA_MAX_M)");
        return 0;
    }
    if (max_iter < 1) {
        fail(GPSPCA_EINVAL, "max_iter must be >= 1");
        return 0;
    }
    int ncu = 0;
    if (device_cus(&ncu) != GPSPCA_OK) return 0;
    const size_t P = (size_t)A->p;
    return deflated_core(A, max_iter, ncu) + al256(sizeof(double) * P * m) +
           al256(sizeof(float) * P) + al256(sizeof(double) * P);
}

int gpspca_solve_deflated(const gpspca_matrix* A, int form, int m, double gamma, double tol,
                          int max_iter, void* workspace, size_t ws_bytes, void* stream, float* X,
                          float* Z, uint32_t* support, double* obj_trace, int* n_iter,
                          int* status) {
    if (form != GPSPCA_SL1 && form != GPSPCA_SL0)
        return fail(GPSPCA_EINVAL, "deflation takes a single-unit formulation");
    int rc = check_problem(A, form, 1, gamma, nullptr);
    if (rc) return rc;
    if (A->dtype != GPSPCA_F32) return fail(GPSPCA_EDTYPE, "deflation runs on FP32 storage");
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    if (!Z || !support || !obj_trace || !n_iter || !status)
        return fail(GPSPCA_EINVAL, "NULL output");
    const size_t need = gpspca_deflated_workspace_bytes(A, m, max_iter);
    if (need == 0) return GPSPCA_EINVAL;
    if (ws_bytes < need) return fail(GPSPCA_ENOMEM, "workspace too small");
    int ncu = 0;
    rc = device_cus(&ncu);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t P = (size_t)A->p;
    const int64_t words = cdiv(A->n, 32);
    // the single-unit solve's workspace, then Q, the start and a scratch vector
    const size_t core = deflated_core(A, max_iter, ncu);
    uint8_t* base = static_cast<uint8_t*>(workspace);
    double* Q = reinterpret_cast<double*>(base + core);
    float* x0 = reinterpret_cast<float*>(base + core + al256(sizeof(double) * P * m));
    double* scratch = reinterpret_cast<double*>(base + core + al256(sizeof(double) * P * m) +
                                                al256(sizeof(float) * P));
    Plan p1;
    make_plan(A, form, 1, max_iter, ncu, &p1);
    int worst = GPSPCA_OK;
    for (int k = 0; k < m; ++k) {
        const float* start = nullptr;
        if (k > 0) {
            // default start of the deflated matrix: its column of largest norm,
            // projected and normalized
            const Ptrs W = carve(p1, workspace);
            const PassParams pp1 = make_params(A, p1, gamma, nullptr);
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2LL * ncu, cdiv(A->n, 4)));
            GPSPCA_HIP(launch_defl_norms(static_cast<const float*>(A->data), A->lda, (int)A->p,
                                         A->n, k, Q, W.norms, grid, st));
            GPSPCA_HIP(launch_topm(p1, W.norms, W.cand_v, W.cand_i, W.idx, st));
            GPSPCA_HIP(launch_gather(p1, pp1, W.idx, W.g64, st));
            GPSPCA_HIP(launch_deflate((int)A->p, k, Q, W.g64, x0, scratch, nullptr, st));
            start = x0;
        }
        rc = solve_core(A, form, 1, gamma, nullptr, nullptr, 0, nullptr, start, tol, max_iter,
                        workspace, core, st, X + (size_t)k * P, Z + (size_t)k * A->n,
                        support + (size_t)k * words, obj_trace + (size_t)k * max_iter,
                        &n_iter[k], nullptr, nullptr, 0, k > 0 ? Q : nullptr, k);
        if (rc < 0) return rc;
        status[k] = rc;
        if (rc > worst) worst = rc;
        GPSPCA_HIP(launch_append_basis((int)A->p, X + (size_t)k * P, Q + (size_t)k * P, st));
    }
    GPSPCA_HIP(hipStreamSynchronize(st));
    if (worst != GPSPCA_OK) g_err = "some component flagged (see status)";
    return worst;
}

int gpspca_refine_path(const gpspca_matrix* A, int form, int K, const double* gammas,
                       const uint32_t* support_in, const float* X0, double tol, int max_iter,
                       void* workspace, size_t ws_bytes, void* stream, float* X, float* Z,
                       uint32_t* support, double* obj_trace, int* n_iter, int* status) {
    int rc = check_path(A, form, K, gammas);
    if (rc) return rc;
    if (A->dtype != GPSPCA_F32) return fail(GPSPCA_EDTYPE, "refinement runs on FP32 storage");
    rc = check_run(tol, max_iter, X, workspace);
    if (rc) return rc;
    if (!support_in) return fail(GPSPCA_EINVAL, "support is NULL");
    if (!X0) return fail(GPSPCA_EINVAL, "refinement needs X0");
    return solve_core(A, form, K, 0.0, nullptr, gammas, 1, support_in, X0, tol, max_iter,
                      workspace, ws_bytes, static_cast<hipStream_t>(stream), X, Z, support,
                      obj_trace, n_iter, status, nullptr);
}

int gpspca_quantize(const gpspca_matrix* A, int to, void* out, int64_t ldq, float* col_scale,
                    void* stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (A->dtype != GPSPCA_F32) return fail(GPSPCA_EDTYPE, "quantize takes an FP32 matrix");
    if (to != GPSPCA_BF16 && to != GPSPCA_F8E4M3)
        return fail(GPSPCA_EDTYPE, "quantize targets BF16 or F8E4M3");
    if (!out) return fail(GPSPCA_EINVAL, "out is NULL");
    if (ldq < A->p) return fail(GPSPCA_EINVAL, "ldq must be >= p");
    if (to == GPSPCA_F8E4M3 && !col_scale)
        return fail(GPSPCA_EINVAL, "F8E4M3 needs col_scale");
    GPSPCA_HIP(launch_quantize(static_cast<const float*>(A->data), A->lda, (int)A->p, A->n, to,
                               out, ldq, col_scale, static_cast<hipStream_t>(stream)));
    return GPSPCA_OK;
}

}  // extern "C"

namespace gpspca {

// Time `passes` passes of configuration `tn` (after one untimed pass) from the
// feasible start X0.  Returns GPSPCA_ENOMEM when the workspace is too small.
static int time_config(const gpspca_matrix* A, int pform, int m, double gamma, int path,
                       const Tune& tn, const float* X0, int passes, void* ws, size_t ws_bytes,
                       hipStream_t st, int ncu, float* ms) {
    Plan pl;
    make_plan(A, pform, m, passes + 1, ncu, &pl, path, 0, &tn);
    if (ws_bytes < pl.total) return GPSPCA_ENOMEM;
    const Ptrs P = carve(pl, ws);
    std::vector<double> gam(m, gamma);
    PassParams pp = make_params(A, pl, gamma, nullptr, path ? gam.data() : nullptr);
    pp.nact = &P.ctrl->nact;
    GPSPCA_HIP(launch_ctrl_reset(P.ctrl, passes + 1, 0.0, st));
    GPSPCA_HIP(launch_fill_zero(P.x[0], sizeof(float) * pl.ldx * pl.mpad, st));
    GPSPCA_HIP(launch_fill_zero(P.x[1], sizeof(float) * pl.ldx * pl.mpad, st));
    if (path) GPSPCA_HIP(launch_fill_zero(P.pstate, sizeof(PathState) * m, st));
    GPSPCA_HIP(launch_load_g64(pl, X0, (int)A->p, P.g64, st));
    if (path) {
        GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 2, P.g64, P.gram, P.ctrl, st));
        GPSPCA_HIP(launch_project_diag(pl, P.gram, P.coef, P.ctrl, st));
    } else {
        GPSPCA_HIP(launch_gram(pl, nullptr, 0, nullptr, 0, P.g64, P.gram, P.ctrl, st));
        GPSPCA_HIP(launch_project(pl, P.gram, P.coef, P.ctrl, st));
    }
    GPSPCA_HIP(launch_apply(pl, P.g64, P.x[1], P.coef, P.x[0], nullptr, P.ctrl, st));
    if (pl.use_mfma || pl.use_q) {
        GPSPCA_HIP(launch_fill_zero(P.xil[1], pl.xil_bytes, st));
        GPSPCA_HIP(launch_x_interleave(pl, P.x[0], P.xil[0], st));
    }
    TimedLaunches tl;
    int rc = enqueue_pass(pl, pp, P, 0, st, tl);
    if (rc) return rc;
    hipEvent_t a = nullptr, b = nullptr;
    GPSPCA_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(GPSPCA_EDEVICE, hipGetErrorString(e));
    }
    e = hipEventRecord(a, st);
    for (int k = 1; k <= passes && e == hipSuccess && rc == GPSPCA_OK; ++k)
        rc = enqueue_pass(pl, pp, P, k, st, tl);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return fail(GPSPCA_EDEVICE, hipGetErrorString(e));
    *ms /= (float)passes;
    return GPSPCA_OK;
}

static std::string tune_text(const Plan& pl) {
    char b[96];
    const char* k = pl.fused_m1 ? "k_pass_m1" : pl.use_vx ? "k_corr_vx"
                  : pl.use_x3 ? "k_corr_x3"
                  : pl.use_rd ? (pl.rd128 ? "k_corr_rd(128-byte lines)" : "k_corr_rd")
                  : pl.use_wg ? "k_corr_wg"
                  : pl.use_qw ? "k_corr_qw"
                  : pl.use_q ? "k_corr_q" : pl.use_mfma ? "k_corr_mfma" : pl.use_mv ? "k_corr_mv"
                  : "k_corr";
    std::snprintf(b, sizeof(b), "%s stages=%d waves_per_cu=%d grid=%d", k,
                  (pl.use_rd || pl.use_x3) ? pl.rd_depth : pl.mfma_stages, pl.waves_per_cu,
                  pl.corr_grid);
    return b;
}

}  // namespace gpspca

extern "C" {

int gpspca_autotune(const gpspca_matrix* A, int form, int m, double gamma, const float* X0,
                    int passes, void* workspace, size_t ws_bytes, void* stream,
                    int* n_timed, double* best_ms, char* best_desc, size_t desc_len) {
    const int path = (form == GPSPCA_SL1 || form == GPSPCA_SL0) && m > 1;
    int rc = path ? check_matrix(A) : check_problem(A, form, m, gamma, nullptr);
    if (rc) return rc;
    if (path && (m > kMaxM || m > A->p)) return fail(GPSPCA_EINVAL, "need K <= GPSPCA_MAX_M and K <= p");
    if (!std::isfinite(gamma) || gamma < 0.0) return fail(GPSPCA_EINVAL, "gamma must be finite and >= 0");
    if (!X0) return fail(GPSPCA_EINVAL, "X0 is NULL");
    if (passes < 1 || passes > 1000) return fail(GPSPCA_EINVAL, "need 1 <= passes <= 1000");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return fail(GPSPCA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    int ncu = 0;
    rc = device_cus(&ncu);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int pform = path ? (form == GPSPCA_SL0 ? GPSPCA_BL0 : GPSPCA_BL1) : form;
    const std::vector<Tune> cand = tune_candidates(A, m, path);
    int timed = 0, best = -1;
    float best_t = 0.f;
    for (size_t i = 0; i < cand.size(); ++i) {
        float t = 0.f;
        rc = time_config(A, pform, m, gamma, path, cand[i], X0, passes, workspace, ws_bytes, st,
                         ncu, &t);
        if (rc == GPSPCA_ENOMEM) continue;
        if (rc) return rc;
        ++timed;
        if (best < 0 || t < best_t) { best = (int)i; best_t = t; }
    }
    if (best < 0) return fail(GPSPCA_ENOMEM, "workspace too small for every configuration");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(A, m, path)] = cand[best];
    }
    Plan pl;
    make_plan(A, pform, m, passes + 1, ncu, &pl, path, 0, &cand[best]);
    if (n_timed) *n_timed = timed;
    if (best_ms) *best_ms = best_t;
    if (best_desc && desc_len) std::snprintf(best_desc, desc_len, "%s", tune_text(pl).c_str());
    return GPSPCA_OK;
}

int gpspca_autotune_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return GPSPCA_OK;
}

int gpspca_column_norms(const gpspca_matrix* A, double* norms, void* stream) {
    int rc = check_matrix(A);
    if (rc) return rc;
    if (!norms) return fail(GPSPCA_EINVAL, "norms is NULL");
    int ncu = 0;
    rc = device_cus(&ncu);
    if (rc) return rc;
    Plan pl;
    make_plan(A, GPSPCA_SL1, 1, 1, ncu, &pl);
    const PassParams pp = make_params(A, pl, 0.0, nullptr);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(2LL * ncu, cdiv(A->n, 16)));
    GPSPCA_HIP(launch_colnorm(pp, A->dtype, norms, grid, static_cast<hipStream_t>(stream)));
    return GPSPCA_OK;
}

int gpspca_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on > 0;
    g_prof.every = on > 0 ? on : 1;
    return GPSPCA_OK;
}

int gpspca_profile_read(double* total_ms, int64_t* launches, char* name, size_t name_len) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (total_ms) *total_ms = g_prof.total_ms;
    if (launches) *launches = g_prof.launches;
    if (name && name_len) {
        std::snprintf(name, name_len, "%s", g_prof.name.c_str());
    }
    g_prof.total_ms = 0.0;
    g_prof.launches = 0;
    return GPSPCA_OK;
}

}  // extern "C"
