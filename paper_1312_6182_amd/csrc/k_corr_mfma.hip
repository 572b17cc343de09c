// Correlation + threshold of the block power iteration on the gfx950 matrix
// cores, with A streamed from HBM into LDS by direct global->LDS DMA.
//
//   Y^T = X^T A,  y_ij = a_i^T x_j  (Table 1), then the soft / hard threshold
//   of each y_ij, S and a per-column activity flag, objective partials.
//
// Work decomposition (one wavefront per workgroup, no barriers):
//   - each wave owns a contiguous range of whole tiles of 16 columns (the
//     same number of tiles, +-1, for every wave) and walks it in chunks of up
//     to 4 or 8 tiles (64 or 128 columns); a shorter last chunk issues DMA and
//     matrix-core work for its own tiles only.  With 8-tile chunks a wave's
//     columns usually fit one chunk, so X is staged once per wave;
//   - the rows of a chunk are streamed in stages of 32 rows: 2 DMA
//     instructions per tile bring the A stage into LDS (column-major, quads
//     XOR-swizzled per column so that the MFMA operand reads are free of bank
//     conflicts), 2 per component block bring the matching X rows;
//     STAGES stages are in flight while the oldest is consumed (X comes from
//     a row-quad-interleaved copy, so each of its DMA instructions reads one
//     contiguous 1 KB);
//   - each stage feeds v_mfma_f32_16x16x4_f32 with M = 16 columns, N = 16
//     components, K = 4 rows: lane l supplies A[row 4(l/16)+t][col l%16] and
//     X[row 4(l/16)+t][comp l%16] for t = 0..3 (one 16-byte LDS read each);
//   - the accumulators hold D[col][comp] (lane l: comp l%16, columns
//     4(l/16)+v), so the threshold runs directly on them.
// LDS reads are issued with inline asm and every wait is explicit, because
// the compiler cannot count LDS DMA completions across the loop back-edge.
#include "gpspca_internal.h"
#include "storage.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <cstdlib>

namespace gpspca {

typedef float f4m __attribute__((ext_vector_type(4)));

namespace {

constexpr int kT = 4;          // column tiles of 16 per chunk
constexpr int kQS = 8;         // row quads per stage (32 rows)

// LDS slot of (column c, quad q) within an A stage: quads are XOR-swizzled by
// bits 1..3 of the column, so that the 16 columns read together by an MFMA
// operand load fall on 16 distinct groups of 4 banks.
__device__ __forceinline__ uint32_t a_slot(int c, int q) {
    return (uint32_t)(16 * (c * kQS + (q ^ ((c >> 1) & 7))));
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ __forceinline__ void wait_lgkm0() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Re-define a register after the preceding (volatile, hence ordered) wait, so
// that its consumers cannot be scheduled before the wait: the output of an
// inline-asm LDS read counts as available as soon as the asm is issued.
__device__ __forceinline__ void after_wait(f4m& v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ f4m lds_read16(uint32_t lds_addr) {
    f4m v;
    asm volatile("ds_read_b128 %0, %1" : "=v"(v) : "v"(lds_addr) : "memory");
    return v;
}

__device__ __forceinline__ void dma16(const float* gptr, uint32_t lds_base) {
    __builtin_amdgcn_global_load_lds(
        (const void __attribute__((address_space(1)))*)gptr,
        (void __attribute__((address_space(3)))*)(uintptr_t)lds_base, 16, 0, 0);
}

__device__ __forceinline__ bool threshold_m(bool l0, double mu, double gamma, float y, float& s,
                                            double& fv) {
    const double yd = (double)y;
    if (l0) {
        const double my = mu * yd;
        const double q = my * my - gamma;
        if (q > 0.0) { s = (float)my; fv = q; return true; }
    } else {
        const double t = mu * fabs(yd) - gamma;
        if (t > 0.0) { s = (float)(yd > 0.0 ? t : -t); fv = t * t; return true; }
    }
    s = 0.f;
    fv = 0.0;
    return false;
}

// Balanced partition: a wave's row-split share of a leftover tile, the 16
// columns from col over the stages s0 .. s1 - 1.  A wave has at most two, and
// their stage ranges are disjoint.
struct XPiece {
    int64_t col;
    int s0, s1;
};

}  // namespace

// One chunk of NT tiles of 16 columns (NT <= 4) starting at column c0: stream
// its rows through the LDS stages, multiply on the matrix cores, threshold.
// Columns at or past cend are clamped to cend - 1 and their results dropped.
// HX (m <= 8, J = 1): X is staged for components 0..7 only, by one DMA
// instruction per stage instead of two; lanes of components 8..15 read the
// same LDS line as component lj - 8, whose products land in outputs that are
// never stored.
// BAL (balanced partition, 2 stages): the chunk also streams the wave's pieces
// of leftover tiles (xp[0 .. nxp-1]) as tile NT of the stages in their ranges,
// and writes their partial sums (the accumulator layout, 1 KB per piece and
// component group) to xout[256 (J e + jb) ..].
template <int NT, int J, int STAGES, int TMAX, bool HX = false, bool BAL_ = false>
__device__ __forceinline__ void mfma_chunk(const PassParams& pp, int64_t c0, int64_t cend,
                                           uint32_t lbase, const float* const* xcol,
                                           const float* __restrict__ Xil, double* f_acc,
                                           int* nnz_acc, float* __restrict__ S,
                                           uint8_t* __restrict__ act,
                                           const XPiece* xp = nullptr, int nxp = 0,
                                           float* __restrict__ xout = nullptr) {
    constexpr bool BAL = BAL_ && NT < TMAX;   // a full chunk never carries pieces
    static_assert(!BAL_ || STAGES == 2, "pieces need 2 stages");
    int nact_l = 0;   // active columns written by this lane
    static_assert(!HX || J == 1, "half X staging needs one component group");
    constexpr int AStage = TMAX * 16 * kQS * 16;   // A bytes per stage: TMAX tiles x 32 rows
    constexpr int XStageBytes = HX ? 1024 : J * 2 * 1024;
    constexpr int StageBytes = AStage + XStageBytes;
    constexpr int ADMA = 2 * NT;           // A DMA instructions per stage (8 columns each)
    constexpr int PER = ADMA + (HX ? 1 : 2 * J);   // DMA instructions per stage
    const int lane = threadIdx.x;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nqf = p >> 2;
    const int nqx = pp.ldx >> 2;           // quads of the X buffers; the last is zero
    const int nst = (nqf + kQS - 1) / kQS;
    const bool l0 = pp.l0 != 0;

    // A DMA sources: slot L = 64 i + lane holds column L / 8 and the quad whose
    // swizzled position is L % 8
    const float* acol[ADMA];
    int aq[ADMA];
#pragma unroll
    for (int i = 0; i < ADMA; ++i) {
        const int L = 64 * i + lane;
        const int cl = L / kQS;
        aq[i] = (L % kQS) ^ ((cl >> 1) & 7);
        int64_t col = c0 + cl;
        col = (col < cend) ? col : cend - 1;
        acol[i] = pp.A + col * pp.lda;
    }
    // pieces: DMA sources laid out as a tile of this chunk (instructions 0, 1
    // of a tile have the swizzled quads aq[0], aq[1]); stage ranges
    // (scalars, not arrays, so that nothing of this lands in scratch or LDS)
    const float *xa00 = pp.A, *xa01 = pp.A, *xa10 = pp.A, *xa11 = pp.A;
    int64_t xc0 = 0, xc1 = 0;
    int xs00 = 0, xs10 = 0, xs01 = 0, xs11 = 0;   // stage range [xs0e, xs1e) of piece e
    if constexpr (BAL) {
        if (nxp > 0) { xc0 = xp[0].col; xs00 = xp[0].s0; xs10 = xp[0].s1; }
        if (nxp > 1) { xc1 = xp[1].col; xs01 = xp[1].s0; xs11 = xp[1].s1; }
        auto src = [&](int64_t base, int ii) {
            int64_t col = base + (64 * ii + lane) / kQS;
            col = (col < pp.n) ? col : pp.n - 1;
            return pp.A + col * pp.lda;
        };
        xa00 = src(xc0, 0);
        xa01 = src(xc0, 1);
        xa10 = src(xc1, 0);
        xa11 = src(xc1, 1);
    }
    // the piece streamed in stage st: 0, 1, or -1 (none)
    auto xpiece = [&](int st) -> int {
        if constexpr (BAL) {
            if (st >= xs00 && st < xs10) return 0;
            if (st >= xs01 && st < xs11) return 1;
        }
        return -1;
    };
    auto issue = [&](int st) {
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
        const int q0 = kQS * st;
#pragma unroll
        for (int i = 0; i < ADMA; ++i) {
            int q = q0 + aq[i];
            q = (q < nqf) ? q : nqf - 1;
            dma16(acol[i] + 4 * q, sb + 1024 * i);
        }
        if constexpr (BAL) {
            const int e = xpiece(st);
            if (e >= 0) {
                int qa = q0 + aq[0], qb = q0 + aq[1];
                qa = (qa < nqf) ? qa : nqf - 1;
                qb = (qb < nqf) ? qb : nqf - 1;
                dma16((e == 0 ? xa00 : xa10) + 4 * qa, sb + 1024 * (2 * NT));
                dma16((e == 0 ? xa01 : xa11) + 4 * qb, sb + 1024 * (2 * NT + 1));
            }
        }
        // X: 4 row quads x 16 components per instruction, one contiguous 1 KB
        // of the interleaved copy (rows past the full quads read the zero quad);
        // HX: 8 row quads x 8 components (lane L: quad L / 8, component L % 8)
        if constexpr (HX) {
            int q = q0 + (lane >> 3);
            q = (q < nqf) ? q : nqx - 1;
            dma16(Xil + ((size_t)q * 16 + (lane & 7)) * 4, sb + AStage);
        } else {
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    int q = q0 + 4 * i + lk;
                    q = (q < nqf) ? q : nqx - 1;
                    dma16(Xil + ((size_t)(jb * nqx + q) * 16 + lj) * 4,
                          sb + AStage + 1024 * (2 * jb + i));
                }
        }
    };

    f4m acc[NT][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4m{0.f, 0.f, 0.f, 0.f};
    f4m accx0[J], accx1[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) accx0[jb] = accx1[jb] = f4m{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
        if (s < nst) issue(s);

    for (int st = 0; st < nst; ++st) {
        if (st + STAGES - 1 < nst) issue(st + STAGES - 1);
        const int ahead = (nst - 1 - st < STAGES - 1) ? nst - 1 - st : STAGES - 1;
        if constexpr (STAGES >= 4) {
            if (ahead >= 3) wait_vmcnt<3 * PER>();
            else if (ahead == 2) wait_vmcnt<2 * PER>();
            else if (ahead == 1) wait_vmcnt<PER>();
            else wait_vmcnt<0>();
        } else if constexpr (STAGES == 3) {
            if (ahead >= 2) wait_vmcnt<2 * PER>();
            else if (ahead == 1) wait_vmcnt<PER>();
            else wait_vmcnt<0>();
        } else {
            // the next stage's instructions may stay in flight (two more when
            // it streams a piece)
            if (ahead >= 1) {
                if (BAL && xpiece(st + 1) >= 0) wait_vmcnt<PER + 2>();
                else wait_vmcnt<PER>();
            } else {
                wait_vmcnt<0>();
            }
        }
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
        const int xe = xpiece(st);
        // both halves of the stage are read before the first multiplies, so the
        // second half's LDS latency hides behind the first half's MFMAs
        f4m av[2][NT], xv[2][J], avx0, avx1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                av[h][t] = lds_read16(sb + a_slot(16 * t + lj, 4 * h + lk));
            if (BAL && xe >= 0) {
                const f4m r = lds_read16(sb + a_slot(16 * NT + lj, 4 * h + lk));
                if (h == 0) avx0 = r;
                else avx1 = r;
            }
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
                xv[h][jb] = HX ? lds_read16(sb + AStage + 16u * (uint32_t)((4 * h + lk) * 8 + (lj & 7)))
                               : lds_read16(sb + AStage + 2048u * jb +
                                            16u * (uint32_t)((4 * h + lk) * 16 + lj));
            if (h == 0) {
                // wait for the first half's reads before the second half's are issued
                wait_lgkm0();
#pragma unroll
                for (int t = 0; t < NT; ++t) after_wait(av[0][t]);
#pragma unroll
                for (int jb = 0; jb < J; ++jb) after_wait(xv[0][jb]);
                if (BAL && xe >= 0) after_wait(avx0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the second half's reads ahead of the MFMAs
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        av[0][t][tm], xv[0][jb][tm], acc[t][jb], 0, 0, 0);
        if (BAL && xe == 0) {
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    accx0[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avx0[tm], xv[0][jb][tm], accx0[jb], 0, 0, 0);
        } else if (BAL && xe == 1) {
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    accx1[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avx0[tm], xv[0][jb][tm], accx1[jb], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);  // the first half's MFMAs stay before the wait
        wait_lgkm0();
#pragma unroll
        for (int t = 0; t < NT; ++t) after_wait(av[1][t]);
#pragma unroll
        for (int jb = 0; jb < J; ++jb) after_wait(xv[1][jb]);
        if (BAL && xe >= 0) after_wait(avx1);
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        av[1][t][tm], xv[1][jb][tm], acc[t][jb], 0, 0, 0);
        if (BAL && xe == 0) {
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    accx0[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avx1[tm], xv[1][jb][tm], accx0[jb], 0, 0, 0);
        } else if (BAL && xe == 1) {
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    accx1[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(avx1[tm], xv[1][jb][tm], accx1[jb], 0, 0, 0);
        }
    }

    // ragged tail rows 4*nqf .. p-1 (p % 4 of them)
    if (p & 3) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t col = c0 + 16 * t + 4 * lk + v;
                col = (col < cend) ? col : cend - 1;
                const float* ac = pp.A + col * pp.lda;
                for (int r = 4 * nqf; r < p; ++r) {
                    const float a = ac[r];
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                }
            }
        // the piece whose range ends at the last stage takes the ragged rows
        if constexpr (BAL) {
            // (at most one piece ends at the last stage: the ranges are disjoint)
            const int eo = (nxp > 0 && xs10 == nst) ? 0 : (nxp > 1 && xs11 == nst) ? 1 : -1;
            if (eo >= 0) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int64_t col = (eo == 0 ? xc0 : xc1) + 4 * lk + v;
                    col = (col < pp.n) ? col : pp.n - 1;
                    const float* ac = pp.A + col * pp.lda;
#pragma unroll
                    for (int jb = 0; jb < J; ++jb) {
                        float sv = eo == 0 ? accx0[jb][v] : accx1[jb][v];
                        for (int r = 4 * nqf; r < p; ++r) sv = __builtin_fmaf(ac[r], xcol[jb][r], sv);
                        if (eo == 0) accx0[jb][v] = sv;
                        else accx1[jb][v] = sv;
                    }
                }
            }
        }
    }
    if constexpr (BAL) {
#pragma unroll
        for (int jb = 0; jb < J; ++jb) {
            if (nxp > 0) *reinterpret_cast<f4m*>(xout + 256 * jb + 4 * lane) = accx0[jb];
            if (nxp > 1) *reinterpret_cast<f4m*>(xout + 256 * (J + jb) + 4 * lane) = accx1[jb];
        }
    }

    // threshold, S, activity flags
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + 16 * t + 4 * lk + v;
            const bool cvalid = col < cend;
            bool any = false;
#pragma unroll
            for (int jb = 0; jb < J; ++jb) {
                const int comp = 16 * jb + lj;
                if (cvalid && comp < m) {
                    float s;
                    double fv;
                    const bool a = threshold_m(l0, pp.mu[comp], pp.gam[comp], acc[t][jb][v], s, fv);
                    S[col * m + comp] = s;
                    if (a) {
                        f_acc[jb] += fv;
                        nnz_acc[jb] += 1;
                        any = true;
                    }
                }
            }
            const uint64_t bal = __ballot(any);
            if (cvalid && lj == 0) {
                const int fl = ((bal >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
                act[col] = fl;
                nact_l += fl;
            }
        }
    add_active_count(nact_l, pp.nact);
}

// J: component blocks of 16 (m <= 16 J);  STAGES: stages in flight.
// TMAX: tiles of 16 columns per chunk (4, or 8 to stage X once per wave when
// a wave owns up to 128 columns).
// BAL: balanced partition (J = 1, 2 stages; bal.q + 1 <= TMAX).  Wave w owns
// the whole tiles q w .. q (w + 1) - 1, and the rem = ntile - q W leftover
// tiles at the end of A are split by row stages over all waves: their
// rem x nst (tile, stage) pairs, tile-major, are cut into W near-equal
// contiguous ranges, so every wave streams the same amount of A up to one
// stage of one tile.  A wave's range covers at most two leftover tiles; their
// partial sums go to bal.xpart[((2 w + piece) J + group) * 256 ..], and k_corr_bal_fix
// finishes those tiles.  Without it, W not dividing ntile leaves some waves a
// whole tile more than others, and they stream it at the end, alone.
template <int J, int STAGES, int TMAX = 4, bool HX = false, bool BAL = false>
__global__ __launch_bounds__(64) void k_corr_mfma(PassParams pp, const float* __restrict__ X,
                                                  const float* __restrict__ Xil,
                                                  float* __restrict__ S,
                                                  uint8_t* __restrict__ act,
                                                  double* __restrict__ fpart,
                                                  int* __restrict__ nnzpart,
                                                  const Ctrl* __restrict__ ctrl, BalArgs bal) {
    if (ctrl->done) return;
    constexpr int XStageBytes = HX ? 1024 : J * 2 * 1024;
    constexpr int StageBytes = TMAX * 16 * kQS * 16 + XStageBytes;
    __shared__ __attribute__((aligned(16))) uint8_t lds[STAGES * StageBytes];
    const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)lds;

    const int lane = threadIdx.x;
    const int m = pp.m, ldx = pp.ldx;
    const int64_t n = pp.n;
    const int64_t W = gridDim.x, w = blockIdx.x;
    // partition in whole tiles of 16 columns: every wave gets the same number
    // of tiles (+-1) and issues DMA and matrix-core work only for those, so no
    // wave streams clamped duplicate columns except in the last tile of A
    const int64_t ntile = (n + 15) / 16;
    int64_t cbeg = 16 * (ntile * w / W);
    int64_t cend = std::min<int64_t>(n, 16 * (ntile * (w + 1) / W));
    XPiece xp[2];
    int nxp = 0;
    if constexpr (BAL) {
        cbeg = 16 * (int64_t)bal.q * w;
        cend = std::min<int64_t>(n, 16 * (int64_t)bal.q * (w + 1));
        const int64_t nst = ((pp.p >> 2) + kQS - 1) / kQS;
        const int64_t R = (int64_t)bal.rem * nst;
        const int64_t a = R * w / W, b = R * (w + 1) / W;
        if (a < b) {
            const int64_t ua = a / nst, t0 = (int64_t)bal.q * W;
            xp[0].col = 16 * (t0 + ua);
            xp[0].s0 = (int)(a - ua * nst);
            xp[0].s1 = (int)std::min<int64_t>(b - ua * nst, nst);
            nxp = 1;
            if (b - ua * nst > nst) {
                xp[1].col = 16 * (t0 + ua + 1);
                xp[1].s0 = 0;
                xp[1].s1 = (int)(b - (ua + 1) * nst);
                nxp = 2;
            }
        }
    }
    const int64_t NW = BAL ? bal.nwp : W;   // objective partial slots per component

    const int lj = lane & 15;

    double f_acc[J];
    int nnz_acc[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) { f_acc[jb] = 0.0; nnz_acc[jb] = 0; }

    // component columns of X (component-major) for the ragged tail rows
    const float* xcol[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) xcol[jb] = X + (size_t)(16 * jb + lj) * ldx;

    for (int64_t c0 = cbeg; c0 < cend; c0 += 16 * TMAX) {
        const int64_t left = cend - c0;
        const int nt = left >= 16 * TMAX ? TMAX : (int)((left + 15) / 16);
#define GPSPCA_CH(NT) mfma_chunk<NT, J, STAGES, TMAX, HX, BAL>(pp, c0, cend, lbase, xcol, Xil, f_acc, nnz_acc, S, act, xp, nxp, bal.xpart + (size_t)w * 512 * J)
        if constexpr (TMAX == 8) {
            switch (nt) {
                case 8: GPSPCA_CH(8); break;
                case 7: GPSPCA_CH(7); break;
                case 6: GPSPCA_CH(6); break;
                case 5: GPSPCA_CH(5); break;
                case 4: GPSPCA_CH(4); break;
                case 3: GPSPCA_CH(3); break;
                case 2: GPSPCA_CH(2); break;
                default: GPSPCA_CH(1); break;
            }
        } else {
            switch (nt) {
                case 4: GPSPCA_CH(4); break;
                case 3: GPSPCA_CH(3); break;
                case 2: GPSPCA_CH(2); break;
                default: GPSPCA_CH(1); break;
            }
        }
#undef GPSPCA_CH
    }

    // per-component totals over the lanes sharing lane % 16 (fixed xor order)
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        double f = f_acc[jb];
        int c = nnz_acc[jb];
        f += __shfl_xor(f, 16, 64);
        c += __shfl_xor(c, 16, 64);
        f += __shfl_xor(f, 32, 64);
        c += __shfl_xor(c, 32, 64);
        const int comp = 16 * jb + lj;
        if (lane < 16 && comp < m) {
            fpart[(int64_t)comp * NW + w] = f;
            nnzpart[(int64_t)comp * NW + w] = c;
        }
    }
}

// Leftover tile u of the balanced partition (one wave per tile): the partial
// sums of its row ranges, in the order of the ranges (ascending wave), then the
// threshold, S, the activity flags and the objective partials at slot W + u,
// as k_corr_mfma does for its own tiles (lane l: component 16 jb + l % 16 of
// group jb < J, columns 4 (l / 16) .. + 3 of the tile).
template <int J>
__global__ __launch_bounds__(64) void k_corr_bal_fix(PassParams pp, BalArgs bal, int W,
                                                     float* __restrict__ S,
                                                     uint8_t* __restrict__ act,
                                                     double* __restrict__ fpart,
                                                     int* __restrict__ nnzpart,
                                                     const Ctrl* __restrict__ ctrl) {
    // the flag is read together with the partial sums (reading stale sums is
    // harmless) and checked before anything is written
    const int done = ctrl->done;
    const int lane = threadIdx.x, lj = lane & 15, lk = lane >> 4;
    const int64_t u = blockIdx.x;
    const int64_t nst = ((pp.p >> 2) + kQS - 1) / kQS;
    const int64_t R = (int64_t)bal.rem * nst;
    const int64_t x0 = u * nst, x1 = x0 + nst;
    // first range holding stage-tile x0: the largest w with R w / W <= x0
    int64_t w = x0 * W / R;
    while (w + 1 < W && R * (w + 1) / W <= x0) ++w;
    while (w > 0 && R * w / W > x0) --w;
    // 16 ranges per round: lane k % 16 works out where range w + k is stored
    // (its loads of all 16 are then issued together and added in range order;
    // ranges past the tile, or empty, re-read range 0 and are not added)
    f4m acc[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) acc[jb] = f4m{0.f, 0.f, 0.f, 0.f};
    for (; w < W && R * w / W < x1; w += 16) {
        const int64_t wk = w + lj;
        const int64_t a = R * wk / W, b = R * (wk + 1) / W;
        const int in_k = (wk < W && a < x1 && a < b) ? 1 : 0;
        const int e_k = (a / nst == u) ? 0 : 1;   // 1: the range began in tile u - 1
        const int at_k = in_k ? (int)((wk * 2 + e_k) * J * 64) : 0;   // in f4m units
        f4m v[16][J];
        int in[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            in[k] = __shfl(in_k, k, 64);
            const int at = __shfl(at_k, k, 64);
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
                v[k][jb] = reinterpret_cast<const f4m*>(bal.xpart)[at + 64 * jb + lane];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k)
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
                if (in[k]) acc[jb] += v[k][jb];
    }
    if (done) return;
    const int64_t n = pp.n, c0 = 16 * ((int64_t)bal.q * W + u);
    const int m = pp.m;
    const bool l0 = pp.l0 != 0;
    double f[J];
    int cnt[J], nact_l = 0;
#pragma unroll
    for (int jb = 0; jb < J; ++jb) { f[jb] = 0.0; cnt[jb] = 0; }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t col = c0 + 4 * lk + v;
        const bool cvalid = col < n;
        bool any = false;
#pragma unroll
        for (int jb = 0; jb < J; ++jb) {
            const int comp = 16 * jb + lj;
            if (cvalid && comp < m) {
                float sv;
                double fv;
                if (threshold_m(l0, pp.mu[comp], pp.gam[comp], acc[jb][v], sv, fv)) {
                    f[jb] += fv;
                    cnt[jb] += 1;
                    any = true;
                }
                S[col * m + comp] = sv;
            }
        }
        const uint64_t bal_bits = __ballot(any);
        if (cvalid && lj == 0) {
            const int fl = ((bal_bits >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
            act[col] = fl;
            nact_l += fl;
        }
    }
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        double fj = f[jb];
        int cj = cnt[jb];
        fj += __shfl_xor(fj, 16, 64);
        cj += __shfl_xor(cj, 16, 64);
        fj += __shfl_xor(fj, 32, 64);
        cj += __shfl_xor(cj, 32, 64);
        const int comp = 16 * jb + lj;
        if (lane < 16 && comp < m) {
            fpart[(int64_t)comp * bal.nwp + W + u] = fj;
            nnzpart[(int64_t)comp * bal.nwp + W + u] = cj;
        }
    }
    add_active_count(nact_l, pp.nact);
}

// ---------------------------------------------------------------------------
// k_corr_wg: the matrix-core correlation with four waves per workgroup that
// stream the same row stages in lockstep (one barrier per stage) over their
// own columns and share each stage of X in LDS, so X costs a quarter of the
// DMA instructions it costs one wave alone.  The workgroup owns whole tiles of
// 16 columns; in each round every wave takes its share (up to TMAX tiles) of
// the round's tiles.  Every wave executes the same barriers, including a wave
// with no tiles in a round.
//   stage: per wave TMAX tiles x 32 rows of A (2 KB per tile), then X (2 KB per
//   component block); per stage, wave w waits for its own DMAs, then the
//   barrier makes everyone's DMAs visible and frees the slot read in the last
//   stage, then w issues its DMAs for the stage STAGES - 1 ahead.
// ---------------------------------------------------------------------------
namespace {
template <int J>
__device__ __forceinline__ void wg_issue_x(const float* __restrict__ Xil, int nqx, int nqf, int q0,
                                           int wv, int lane, uint32_t xbase) {
    const int lj = lane & 15, lk = lane >> 4;
    if constexpr (J == 1) {
        // two 1 KB instructions: wave w moves half of instruction w / 2
        const int i = wv >> 1;
        if ((lane >> 5) == (wv & 1)) {
            int q = q0 + 4 * i + lk;
            q = (q < nqf) ? q : nqx - 1;
            dma16(Xil + ((size_t)q * 16 + lj) * 4, xbase + 1024 * i);
        }
    } else {
#pragma unroll
        for (int u = 0; u < J / 2; ++u) {
            const int idx = wv + 4 * u;          // instruction idx = 2 jb + i
            const int jb = idx >> 1, i = idx & 1;
            int q = q0 + 4 * i + lk;
            q = (q < nqf) ? q : nqx - 1;
            dma16(Xil + ((size_t)(jb * nqx + q) * 16 + lj) * 4, xbase + 2048u * jb + 1024 * i);
        }
    }
}
}  // namespace

// One round of a wave that owns NT tiles (NT = 0: it only helps with X).
template <int NT, int J, int STAGES, int TMAX>
__device__ __forceinline__ void wg_round(const PassParams& pp, int64_t c0, int64_t cend,
                                         uint32_t lbase, int wv, const float* const* xcol,
                                         const float* __restrict__ Xil, double* f_acc,
                                         int* nnz_acc, float* __restrict__ S,
                                         uint8_t* __restrict__ act) {
    int nact_l = 0;   // active columns written by this lane
    constexpr int AW = TMAX * 2048;                 // A bytes per wave per stage
    constexpr int StageBytes = 4 * AW + J * 2048;
    constexpr int ADMA = 2 * NT;
    constexpr int XW = (J == 1) ? 1 : J / 2;        // X DMA instructions per wave
    constexpr int PER = ADMA + XW;
    const int lane = threadIdx.x & 63;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nqf = p >> 2;
    const int nqx = pp.ldx >> 2;
    const int nst = (nqf + kQS - 1) / kQS;
    const bool l0 = pp.l0 != 0;

    const float* acol[ADMA > 0 ? ADMA : 1];
    int aq[ADMA > 0 ? ADMA : 1];
#pragma unroll
    for (int i = 0; i < ADMA; ++i) {
        const int L = 64 * i + lane;
        const int cl = L / kQS;
        aq[i] = (L % kQS) ^ ((cl >> 1) & 7);
        int64_t col = c0 + cl;
        col = (col < cend) ? col : cend - 1;
        acol[i] = pp.A + col * pp.lda;
    }
    auto issue = [&](int st) {
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
        const int q0 = kQS * st;
#pragma unroll
        for (int i = 0; i < ADMA; ++i) {
            int q = q0 + aq[i];
            q = (q < nqf) ? q : nqf - 1;
            dma16(acol[i] + 4 * q, sb + wv * AW + 1024 * i);
        }
        wg_issue_x<J>(Xil, nqx, nqf, q0, wv, lane, sb + 4 * AW);
    };

    f4m acc[NT > 0 ? NT : 1][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4m{0.f, 0.f, 0.f, 0.f};

    // the previous round's last stage may still be read by other waves
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < STAGES - 1; ++s2)
        if (s2 < nst) issue(s2);

    for (int st = 0; st < nst; ++st) {
        // own DMAs of stage st done: later stages issued so far are st+1 .. st+STAGES-2
        const int later = (nst - 1 - st < STAGES - 2) ? nst - 1 - st : STAGES - 2;
        if constexpr (STAGES >= 4) {
            if (later >= 2) wait_vmcnt<2 * PER>();
            else if (later == 1) wait_vmcnt<PER>();
            else wait_vmcnt<0>();
        } else if constexpr (STAGES == 3) {
            if (later >= 1) wait_vmcnt<PER>();
            else wait_vmcnt<0>();
        } else {
            wait_vmcnt<0>();
        }
        __syncthreads();
        if (st + STAGES - 1 < nst) issue(st + STAGES - 1);
        if constexpr (NT > 0) {
            const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
            const uint32_t sa = sb + wv * AW, sx = sb + 4 * AW;
            f4m av[2][NT], xv[2][J];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    av[h][t] = lds_read16(sa + a_slot(16 * t + lj, 4 * h + lk));
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    xv[h][jb] = lds_read16(sx + 2048u * jb + 16u * (uint32_t)((4 * h + lk) * 16 + lj));
                if (h == 0) {
                    wait_lgkm0();
#pragma unroll
                    for (int t = 0; t < NT; ++t) after_wait(av[0][t]);
#pragma unroll
                    for (int jb = 0; jb < J; ++jb) after_wait(xv[0][jb]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            av[0][t][tm], xv[0][jb][tm], acc[t][jb], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            wait_lgkm0();
#pragma unroll
            for (int t = 0; t < NT; ++t) after_wait(av[1][t]);
#pragma unroll
            for (int jb = 0; jb < J; ++jb) after_wait(xv[1][jb]);
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            av[1][t][tm], xv[1][jb][tm], acc[t][jb], 0, 0, 0);
        }
    }

    if constexpr (NT > 0) {
        if (p & 3) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int64_t col = c0 + 16 * t + 4 * lk + v;
                    col = (col < cend) ? col : cend - 1;
                    const float* ac = pp.A + col * pp.lda;
                    for (int r = 4 * nqf; r < p; ++r) {
                        const float a = ac[r];
#pragma unroll
                        for (int jb = 0; jb < J; ++jb)
                            acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                    }
                }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t col = c0 + 16 * t + 4 * lk + v;
                const bool cvalid = col < cend;
                bool any = false;
#pragma unroll
                for (int jb = 0; jb < J; ++jb) {
                    const int comp = 16 * jb + lj;
                    if (cvalid && comp < m) {
                        float s;
                        double fv;
                        const bool a = threshold_m(l0, pp.mu[comp], pp.gam[comp], acc[t][jb][v], s, fv);
                        S[col * m + comp] = s;
                        if (a) {
                            f_acc[jb] += fv;
                            nnz_acc[jb] += 1;
                            any = true;
                        }
                    }
                }
                const uint64_t bal = __ballot(any);
                if (cvalid && lj == 0) {
                const int fl = ((bal >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
                act[col] = fl;
                nact_l += fl;
            }
            }
    }
    add_active_count(nact_l, pp.nact);
}

template <int J, int STAGES, int TMAX>
__global__ __launch_bounds__(256) void k_corr_wg(PassParams pp, const float* __restrict__ X,
                                                 const float* __restrict__ Xil,
                                                 float* __restrict__ S, uint8_t* __restrict__ act,
                                                 double* __restrict__ fpart,
                                                 int* __restrict__ nnzpart,
                                                 const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int StageBytes = 4 * TMAX * 2048 + J * 2048;
    __shared__ __attribute__((aligned(16))) uint8_t lds[STAGES * StageBytes];
    const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)lds;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = pp.m, ldx = pp.ldx;
    const int64_t n = pp.n;
    const int64_t G = gridDim.x, g = blockIdx.x;
    const int64_t ntile = (n + 15) / 16;
    const int64_t tb = ntile * g / G, te = ntile * (g + 1) / G;   // this workgroup's tiles
    const int lj = lane & 15;

    double f_acc[J];
    int nnz_acc[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) { f_acc[jb] = 0.0; nnz_acc[jb] = 0; }
    const float* xcol[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) xcol[jb] = X + (size_t)(16 * jb + lj) * ldx;

    for (int64_t r0 = tb; r0 < te; r0 += 4 * TMAX) {
        // tiles r0 .. r1-1 of this iteration, split evenly over the four waves
        const int64_t r1 = (r0 + 4 * TMAX < te) ? r0 + 4 * TMAX : te;
        const int64_t nt = r1 - r0;
        const int64_t w0 = r0 + nt * wv / 4, w1 = r0 + nt * (wv + 1) / 4;
        const int64_t c0 = 16 * w0;
        const int64_t cend = std::min<int64_t>(n, 16 * w1);
        const int k = (int)(w1 - w0);
#define GPSPCA_WG(NT) wg_round<NT, J, STAGES, TMAX>(pp, c0, cend, lbase, wv, xcol, Xil, f_acc, nnz_acc, S, act)
        switch (k) {
            case 0: GPSPCA_WG(0); break;
            case 1: GPSPCA_WG(1); break;
            case 2: GPSPCA_WG(2); break;
            case 3: GPSPCA_WG(3); break;
            case 4: GPSPCA_WG(4); break;
            case 5: if constexpr (TMAX >= 5) GPSPCA_WG(5); break;
            case 6: if constexpr (TMAX >= 6) GPSPCA_WG(6); break;
            case 7: if constexpr (TMAX >= 7) GPSPCA_WG(7); break;
            default: if constexpr (TMAX >= 8) GPSPCA_WG(8); break;
        }
#undef GPSPCA_WG
    }

    const int64_t W = G * 4, w = g * 4 + wv;
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        double f = f_acc[jb];
        int c = nnz_acc[jb];
        f += __shfl_xor(f, 16, 64);
        c += __shfl_xor(c, 16, 64);
        f += __shfl_xor(f, 32, 64);
        c += __shfl_xor(c, 32, 64);
        const int comp = 16 * jb + lj;
        if (lane < 16 && comp < m) {
            fpart[(int64_t)comp * W + w] = f;
            nnzpart[(int64_t)comp * W + w] = c;
        }
    }
}

hipError_t launch_corr_wg(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    const dim3 grid(pl.corr_grid), block(256);
#define GPSPCA_KW(JJ, SS, TT) \
    GPSPCA_LAUNCH_TIMED((k_corr_wg<JJ, SS, TT>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl)
    if (pl.m <= 16) {
        if (pl.mfma_stages == 4) GPSPCA_KW(1, 4, 4);
        else GPSPCA_KW(1, 2, 8);
    } else if (pl.m <= 32) {
        GPSPCA_KW(2, 2, 8);
    } else {
        GPSPCA_KW(4, 2, 8);
    }
#undef GPSPCA_KW
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_corr_rd: the same matrix-core correlation with every operand loaded
// straight into registers (no LDS): lane (lj, lk) loads rows 4(4h + lk) ..
// +3 of column 16t + lj (one 16-byte load feeds four MFMAs) and the matching
// X quad of component lj from the interleaved copy.  Stages of 32 rows are
// software-pipelined D deep with compile-time buffer indices; loads past the
// last full quad are clamped and meet zero rows of X, so no load is
// conditional and the compiler's waits stay exact.
// ---------------------------------------------------------------------------
// W128: a load instruction covers 8 columns x 128 bytes (whole cache lines)
// instead of 16 columns x 64 bytes.  Lane l then holds quad 8 st + (l >> 3) of
// column 16 t + (l & 7) (first load) and of column 16 t + 8 + (l & 7) (second
// load); the MFMA operand of lane (lj, lk) for k-slot quad 8 st + 2 lk + hh is
// rebuilt in registers with one swap of the lane halves of each 16-lane row
// (DPP row rotation by 8) and two selects.
__device__ __forceinline__ float swap_row_halves(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false));
}

template <int NT, int J, int D, bool W128>
__device__ __forceinline__ void rd_chunk(const PassParams& pp, int64_t c0, int64_t cend,
                                         const float* const* xcol,
                                         const float* __restrict__ Xil, double* f_acc,
                                         int* nnz_acc, float* __restrict__ S,
                                         uint8_t* __restrict__ act) {
    int nact_l = 0;   // active columns written by this lane
    const int lane = threadIdx.x;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nqf = p >> 2;
    const int nqx = pp.ldx >> 2;
    const int nst = (nqf + kQS - 1) / kQS;
    const bool l0 = pp.l0 != 0;

    constexpr int NH = W128 ? 2 : 1;
    const float* colp[NT][NH];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            int64_t col = W128 ? c0 + 16 * t + 8 * h + (lane & 7) : c0 + 16 * t + lj;
            col = (col < cend) ? col : cend - 1;
            colp[t][h] = pp.A + col * pp.lda;
        }
    const bool lo8 = (lane & 8) == 0;
    f4m abuf[D][NT][2], xbuf[D][J][2];
    auto load = [&](int st, f4m(&ab)[NT][2], f4m(&xb)[J][2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // A: W128 lane quad 8 st + (l >> 3) of column half h; else quad 8 st + 4 h + lk
            const int q = W128 ? kQS * st + (lane >> 3) : kQS * st + 4 * h + lk;
            const int qa = (q < nqf) ? q : nqf - 1;
            // X: the quad of k-slot lk in operand h (8 st + 2 lk + h under W128)
            const int qk = W128 ? kQS * st + 2 * lk + h : q;
            const int qx = (qk < nqf) ? qk : nqx - 1;
#pragma unroll
            for (int t = 0; t < NT; ++t)
                ab[t][h] = __builtin_nontemporal_load(
                    reinterpret_cast<const f4m*>(colp[t][W128 ? h : 0] + 4 * qa));
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
                xb[jb][h] = *reinterpret_cast<const f4m*>(
                    Xil + ((size_t)(jb * nqx + qx) * 16 + lj) * 4);
        }
    };
    f4m acc[NT][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4m{0.f, 0.f, 0.f, 0.f};

    // the scheduling barriers keep every prefetch where it is written (D stages
    // ahead of its use); left alone, the scheduler sinks loads next to their
    // consumers and the pipeline collapses into load-wait-compute
    if (nst > 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) load(d, abuf[d], xbuf[d]);
        __builtin_amdgcn_sched_barrier(0);
        for (int s0 = 0; s0 < nst; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if constexpr (W128) {
                    // operand 0: own first load (lj < 8) or the partner lane's second;
                    // operand 1: the partner's first load (lj < 8) or own second
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int tm = 0; tm < 4; ++tm) {
                            const float a0 = abuf[d][t][0][tm], a1 = abuf[d][t][1][tm];
                            const float sw = swap_row_halves(lo8 ? a1 : a0);
                            abuf[d][t][0][tm] = lo8 ? a0 : sw;
                            abuf[d][t][1][tm] = lo8 ? sw : a1;
                        }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                        for (int t = 0; t < NT; ++t)
#pragma unroll
                            for (int jb = 0; jb < J; ++jb)
                                acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                    abuf[d][t][h][tm], xbuf[d][jb][h][tm], acc[t][jb], 0, 0, 0);
                // stages past the last one re-read it (clamped) and meet zero X
                int nxt = s0 + d + D;
                nxt = (nxt < nst) ? nxt : nst;
                __builtin_amdgcn_sched_barrier(0);
                load(nxt, abuf[d], xbuf[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    if (p & 3) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t col = c0 + 16 * t + 4 * lk + v;
                col = (col < cend) ? col : cend - 1;
                const float* ac = pp.A + col * pp.lda;
                for (int r = 4 * nqf; r < p; ++r) {
                    const float a = ac[r];
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                }
            }
    }

#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + 16 * t + 4 * lk + v;
            const bool cvalid = col < cend;
            bool any = false;
#pragma unroll
            for (int jb = 0; jb < J; ++jb) {
                const int comp = 16 * jb + lj;
                if (cvalid && comp < m) {
                    float s;
                    double fv;
                    const bool a = threshold_m(l0, pp.mu[comp], pp.gam[comp], acc[t][jb][v], s, fv);
                    S[col * m + comp] = s;
                    if (a) {
                        f_acc[jb] += fv;
                        nnz_acc[jb] += 1;
                        any = true;
                    }
                }
            }
            const uint64_t bal = __ballot(any);
            if (cvalid && lj == 0) {
                const int fl = ((bal >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
                act[col] = fl;
                nact_l += fl;
            }
        }
    add_active_count(nact_l, pp.nact);
}

template <int J, int D, bool W128>
__global__ __launch_bounds__(64) void k_corr_rd(PassParams pp, const float* __restrict__ X,
                                                const float* __restrict__ Xil,
                                                float* __restrict__ S, uint8_t* __restrict__ act,
                                                double* __restrict__ fpart,
                                                int* __restrict__ nnzpart,
                                                const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    const int lane = threadIdx.x;
    const int m = pp.m, ldx = pp.ldx;
    const int64_t n = pp.n;
    const int64_t W = gridDim.x, w = blockIdx.x;
    const int64_t ntile = (n + 15) / 16;
    const int64_t cbeg = 16 * (ntile * w / W);
    const int64_t cend = std::min<int64_t>(n, 16 * (ntile * (w + 1) / W));
    const int lj = lane & 15;
    double f_acc[J];
    int nnz_acc[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) { f_acc[jb] = 0.0; nnz_acc[jb] = 0; }
    const float* xcol[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) xcol[jb] = X + (size_t)(16 * jb + lj) * ldx;
    for (int64_t c0 = cbeg; c0 < cend; c0 += 16 * kT) {
        const int64_t left = cend - c0;
        if (left > 48) rd_chunk<4, J, D, W128>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else if (left > 32) rd_chunk<3, J, D, W128>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else if (left > 16) rd_chunk<2, J, D, W128>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else rd_chunk<1, J, D, W128>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
    }
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        double f = f_acc[jb];
        int c = nnz_acc[jb];
        f += __shfl_xor(f, 16, 64);
        c += __shfl_xor(c, 16, 64);
        f += __shfl_xor(f, 32, 64);
        c += __shfl_xor(c, 32, 64);
        const int comp = 16 * jb + lj;
        if (lane < 16 && comp < m) {
            fpart[(int64_t)comp * W + w] = f;
            nnzpart[(int64_t)comp * W + w] = c;
        }
    }
}

hipError_t launch_corr_rd(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    const dim3 grid(pl.corr_grid), block(64);
    const int D = pl.rd_depth;
#define GPSPCA_RD(JJ, DD, WW) \
    GPSPCA_LAUNCH_TIMED((k_corr_rd<JJ, DD, WW>), grid, block, 0, st, pp, X, Xil, S, act, fpart, \
                       nnzpart, ctrl)
#define GPSPCA_RDW(JJ, DD) \
    do { if (pl.rd128) GPSPCA_RD(JJ, DD, true); else GPSPCA_RD(JJ, DD, false); } while (0)
    if (pl.m <= 16) {
        if (D == 2) GPSPCA_RDW(1, 2);
        else if (D == 3) GPSPCA_RDW(1, 3);
        else if (D == 6) GPSPCA_RDW(1, 6);
        else GPSPCA_RDW(1, 4);
    } else if (pl.m <= 32) {
        if (D <= 2) GPSPCA_RDW(2, 2);
        else GPSPCA_RDW(2, 3);
    } else {
        GPSPCA_RDW(4, 2);
    }
#undef GPSPCA_RDW
#undef GPSPCA_RD
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_corr_x3: the correlation of FP32 A and X on the bfloat16 matrix cores.
// Every FP32 value v splits exactly into three bfloat16 parts, v = v1 + v2 +
// v3 (v1 = bf16(v), v2 = bf16(v - v1), v3 = v - v1 - v2: 8 + 8 + 8 bits of
// the 24-bit significand, each residual exact in FP32), and y_ij = a_i^T x_j
// is accumulated in FP32 from the six part products a_k x_l with k + l <= 4.
// The three dropped ones (k + l >= 5) add up to less than 2^-23 |a_ri x_rj|
// per row, the size of FP32's own rounding of the product.  A 16x16x32
// bfloat16 MFMA does 8 times the work of a 16x16x4 FP32 one at twice its
// rate, so the six cost 3/8 of the FP32 matrix-core time: at 64 components,
// where the FP32 kernels are bound by the matrix cores, this one is bound by
// HBM and the splitting (VALU) instead.
// Loads as in k_corr_rd (registers only, software-pipelined D stages of 32
// rows): lane (lj, lk) holds quads lk and 4 + lk of a stage of column 16 t +
// lj, which are the 8 k-values of its bfloat16 operand, and the same quads of
// component lj of X from the interleaved copy.
// ---------------------------------------------------------------------------
typedef __bf16 bf8m __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3_bf16(const f4m& q0, const f4m& q1, bf8m& v1, bf8m& v2,
                                            bf8m& v3) {
    float r[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        r[e] = q0[e];
        r[4 + e] = q1[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        v1[e] = (__bf16)r[e];
        r[e] -= (float)v1[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        v2[e] = (__bf16)r[e];
        r[e] -= (float)v2[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) v3[e] = (__bf16)r[e];
}

template <int NT, int J, int D>
__device__ __forceinline__ void x3_chunk(const PassParams& pp, int64_t c0, int64_t cend,
                                         const float* const* xcol,
                                         const float* __restrict__ Xil, double* f_acc,
                                         int* nnz_acc, float* __restrict__ S,
                                         uint8_t* __restrict__ act) {
    int nact_l = 0;   // active columns written by this lane
    const int lane = threadIdx.x;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nqf = p >> 2;
    const int nqx = pp.ldx >> 2;
    const int nst = (nqf + kQS - 1) / kQS;
    const bool l0 = pp.l0 != 0;

    const float* colp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        int64_t col = c0 + 16 * t + lj;
        col = (col < cend) ? col : cend - 1;
        colp[t] = pp.A + col * pp.lda;
    }
    f4m abuf[D][NT][2], xbuf[D][J][2];
    auto load = [&](int st, f4m(&ab)[NT][2], f4m(&xb)[J][2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = kQS * st + 4 * h + lk;
            const int qa = (q < nqf) ? q : nqf - 1;
            const int qx = (q < nqf) ? q : nqx - 1;   // the last quad of X is zero
#pragma unroll
            for (int t = 0; t < NT; ++t)
                ab[t][h] = __builtin_nontemporal_load(reinterpret_cast<const f4m*>(colp[t] + 4 * qa));
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
                xb[jb][h] = *reinterpret_cast<const f4m*>(
                    Xil + ((size_t)(jb * nqx + qx) * 16 + lj) * 4);
        }
    };
    f4m acc[NT][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4m{0.f, 0.f, 0.f, 0.f};

    if (nst > 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) load(d, abuf[d], xbuf[d]);
        __builtin_amdgcn_sched_barrier(0);
        for (int s0 = 0; s0 < nst; s0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                bf8m x1[J], x2[J], x3[J];
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
                    split3_bf16(xbuf[d][jb][0], xbuf[d][jb][1], x1[jb], x2[jb], x3[jb]);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    bf8m a1, a2, a3;
                    split3_bf16(abuf[d][t][0], abuf[d][t][1], a1, a2, a3);
#pragma unroll
                    for (int jb = 0; jb < J; ++jb) {
                        // smallest terms first
                        f4m c = acc[t][jb];
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, x1[jb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, x2[jb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x3[jb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, x1[jb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x2[jb], c, 0, 0, 0);
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, x1[jb], c, 0, 0, 0);
                    }
                }
                // stages past the last one re-read it (clamped) and meet zero X
                int nxt = s0 + d + D;
                nxt = (nxt < nst) ? nxt : nst;
                __builtin_amdgcn_sched_barrier(0);
                load(nxt, abuf[d], xbuf[d]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    if (p & 3) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t col = c0 + 16 * t + 4 * lk + v;
                col = (col < cend) ? col : cend - 1;
                const float* ac = pp.A + col * pp.lda;
                for (int r = 4 * nqf; r < p; ++r) {
                    const float a = ac[r];
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                }
            }
    }

#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + 16 * t + 4 * lk + v;
            const bool cvalid = col < cend;
            bool any = false;
#pragma unroll
            for (int jb = 0; jb < J; ++jb) {
                const int comp = 16 * jb + lj;
                if (cvalid && comp < m) {
                    float s;
                    double fv;
                    const bool a = threshold_m(l0, pp.mu[comp], pp.gam[comp], acc[t][jb][v], s, fv);
                    S[col * m + comp] = s;
                    if (a) {
                        f_acc[jb] += fv;
                        nnz_acc[jb] += 1;
                        any = true;
                    }
                }
            }
            const uint64_t bal = __ballot(any);
            if (cvalid && lj == 0) {
                const int fl = ((bal >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
                act[col] = fl;
                nact_l += fl;
            }
        }
    add_active_count(nact_l, pp.nact);
}

template <int J, int D>
__global__ __launch_bounds__(64) void k_corr_x3(PassParams pp, const float* __restrict__ X,
                                                const float* __restrict__ Xil,
                                                float* __restrict__ S, uint8_t* __restrict__ act,
                                                double* __restrict__ fpart,
                                                int* __restrict__ nnzpart,
                                                const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    const int lane = threadIdx.x;
    const int m = pp.m, ldx = pp.ldx;
    const int64_t n = pp.n;
    const int64_t W = gridDim.x, w = blockIdx.x;
    const int64_t ntile = (n + 15) / 16;
    const int64_t cbeg = 16 * (ntile * w / W);
    const int64_t cend = std::min<int64_t>(n, 16 * (ntile * (w + 1) / W));
    const int lj = lane & 15;
    double f_acc[J];
    int nnz_acc[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) { f_acc[jb] = 0.0; nnz_acc[jb] = 0; }
    const float* xcol[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) xcol[jb] = X + (size_t)(16 * jb + lj) * ldx;
    for (int64_t c0 = cbeg; c0 < cend; c0 += 16 * kT) {
        const int64_t left = cend - c0;
        if (left > 48) x3_chunk<4, J, D>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else if (left > 32) x3_chunk<3, J, D>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else if (left > 16) x3_chunk<2, J, D>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
        else x3_chunk<1, J, D>(pp, c0, cend, xcol, Xil, f_acc, nnz_acc, S, act);
    }
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        double f = f_acc[jb];
        int c = nnz_acc[jb];
        f += __shfl_xor(f, 16, 64);
        c += __shfl_xor(c, 16, 64);
        f += __shfl_xor(f, 32, 64);
        c += __shfl_xor(c, 32, 64);
        const int comp = 16 * jb + lj;
        if (lane < 16 && comp < m) {
            fpart[(int64_t)comp * W + w] = f;
            nnzpart[(int64_t)comp * W + w] = c;
        }
    }
}

hipError_t launch_corr_x3(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    const dim3 grid(pl.corr_grid), block(64);
#define GPSPCA_X3(JJ, DD) \
    GPSPCA_LAUNCH_TIMED((k_corr_x3<JJ, DD>), grid, block, 0, st, pp, X, Xil, S, act, fpart, \
                       nnzpart, ctrl)
    const bool d3 = pl.rd_depth == 3;
    if (pl.m <= 16) {
        if (d3) GPSPCA_X3(1, 3); else GPSPCA_X3(1, 2);
    } else if (pl.m <= 32) {
        if (d3) GPSPCA_X3(2, 3); else GPSPCA_X3(2, 2);
    } else {
        if (d3) GPSPCA_X3(4, 3); else GPSPCA_X3(4, 2);
    }
#undef GPSPCA_X3
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_corr_mv: the same matrix-core correlation for m <= 16, but A is staged
// through registers instead of LDS DMA: one wave per SIMD can hold three
// 16 KB stages in flight (A streamed as contiguous 512-byte column segments,
// one per half-wave), and LDS only transposes the stage being consumed into
// MFMA operand order.  All loads are ordinary vector loads, so the compiler
// inserts every wait itself.
//   chunk = 32 columns (2 MFMA tiles); stage = 128 rows (32 quads);
//   LDS slot of (column i, quad q): i*512 + 16*(q ^ (i & 31)) (conflict-free
//   for both the half-wave row writes and the 16-column operand reads).
// ---------------------------------------------------------------------------
namespace {
constexpr int kMvQ = 32;   // quads per stage
constexpr int kMvC = 32;   // columns per chunk

__device__ __forceinline__ uint32_t mv_slot(int i, int q) {
    return (uint32_t)(i * 512 + 16 * (q ^ (i & 31)));
}
}  // namespace

__global__ __launch_bounds__(64) void k_corr_mv(PassParams pp, const float* __restrict__ X,
                                                float* __restrict__ S, uint8_t* __restrict__ act,
                                                double* __restrict__ fpart,
                                                int* __restrict__ nnzpart,
                                                const Ctrl* __restrict__ ctrl) {
    int nact_l = 0;   // active columns written by this lane
    if (ctrl->done) return;
    __shared__ __attribute__((aligned(16))) f4m tr[kMvC * kMvQ];  // 16 KB transpose buffer
    const int lane = threadIdx.x;
    const int p = pp.p, m = pp.m, ldx = pp.ldx;
    const int nqf = p >> 2;
    const int rem = p & 3;
    const int nst = (nqf + kMvQ - 1) / kMvQ;
    const bool l0 = pp.l0 != 0;
    const int64_t n = pp.n;
    const int64_t W = gridDim.x, w = blockIdx.x;
    const int64_t cbeg = n * w / W;
    const int64_t cend = n * (w + 1) / W;
    const int lj = lane & 15, lk = lane >> 4;
    const int half = lane >> 5, lq = lane & 31;
    const float* xcol = X + (size_t)lj * ldx;
    const int xzero = ldx - 4;
    double f_acc = 0.0;
    int nnz_acc = 0;
    char* trb = reinterpret_cast<char*>(tr);

    for (int64_t c0 = cbeg; c0 < cend; c0 += kMvC) {
        const float* colp[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            int64_t col = c0 + 2 * c + half;
            col = (col < cend) ? col : cend - 1;
            colp[c] = pp.A + col * pp.lda;
        }
        auto load = [&](int st, f4m(&Ab)[16], f4m(&Xb)[8]) {
            int q = kMvQ * st + lq;
            q = (q < nqf) ? q : nqf - 1;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                Ab[c] = __builtin_nontemporal_load(reinterpret_cast<const f4m*>(colp[c] + 4 * q));
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int qx = kMvQ * st + 4 * g + lk;
                Xb[g] = *reinterpret_cast<const f4m*>(xcol + ((qx < nqf) ? 4 * qx : xzero));
            }
        };
        f4m acc[2];
        acc[0] = f4m{0.f, 0.f, 0.f, 0.f};
        acc[1] = f4m{0.f, 0.f, 0.f, 0.f};
        auto process = [&](const f4m(&Ab)[16], const f4m(&Xb)[8]) {
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const int i = 2 * c + half;
                *reinterpret_cast<f4m*>(trb + mv_slot(i, lq)) = Ab[c];
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const f4m a0 = *reinterpret_cast<const f4m*>(trb + mv_slot(lj, 4 * g + lk));
                const f4m a1 = *reinterpret_cast<const f4m*>(trb + mv_slot(16 + lj, 4 * g + lk));
#pragma unroll
                for (int tm = 0; tm < 4; ++tm) {
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[tm], Xb[g][tm], acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[tm], Xb[g][tm], acc[1], 0, 0, 0);
                }
            }
        };
        // Three register stages in flight.  Loads and stages are unconditional so
        // that the compiler can count the outstanding loads exactly (a stage past
        // the last one loads clamped, already-cached addresses and pairs them with
        // the zero quad of X, so it adds exactly 0).
        f4m A0[16], A1[16], A2[16], X0[8], X1[8], X2[8];
        if (nst > 0) {
            load(0, A0, X0);
            load(1, A1, X1);
            for (int st = 0; st < nst; st += 3) {
                load(st + 2, A2, X2);
                process(A0, X0);
                load(st + 3, A0, X0);
                process(A1, X1);
                load(st + 4, A1, X1);
                process(A2, X2);
            }
        }

        // ragged tail rows 4*nqf .. p-1
        if (rem) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int64_t col = c0 + 16 * t + 4 * lk + v;
                    col = (col < cend) ? col : cend - 1;
                    const float* ac = pp.A + col * pp.lda;
                    for (int r = 4 * nqf; r < p; ++r)
                        acc[t][v] = __builtin_fmaf(ac[r], xcol[r], acc[t][v]);
                }
        }
        // threshold, S, activity flags (lane: component lj, columns 16t + 4lk + v)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t col = c0 + 16 * t + 4 * lk + v;
                const bool valid = col < cend && lj < m;
                bool a = false;
                if (valid) {
                    float sv;
                    double fv;
                    a = threshold_m(l0, pp.mu[lj], pp.gam[lj], acc[t][v], sv, fv);
                    S[col * m + lj] = sv;
                    if (a) {
                        f_acc += fv;
                        nnz_acc += 1;
                    }
                }
                const uint64_t bal = __ballot(a);
                if (col < cend && lj == 0) {
                    const int fl = ((bal >> (16 * lk)) & 0xFFFFull) ? 1 : 0;
                    act[col] = fl;
                    nact_l += fl;
                }
            }
    }
    f_acc += __shfl_xor(f_acc, 16, 64);
    nnz_acc += __shfl_xor(nnz_acc, 16, 64);
    f_acc += __shfl_xor(f_acc, 32, 64);
    nnz_acc += __shfl_xor(nnz_acc, 32, 64);
    if (lane < 16 && lj < m) {
        fpart[(int64_t)lj * W + w] = f_acc;
        nnzpart[(int64_t)lj * W + w] = nnz_acc;
    }
    add_active_count(nact_l, pp.nact);
}

hipError_t launch_corr_mv(const Plan& pl, const PassParams& pp, const float* X, float* S,
                          uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    GPSPCA_LAUNCH_TIMED(k_corr_mv, dim3(pl.corr_grid), dim3(64), 0, st, pp, X, S, act, fpart,
                       nnzpart, ctrl);
    return hipGetLastError();
}

// Resident workgroups per CU of the matrix-core kernel for (m, stages): what
// LDS allows (the caller caps it).
// Half X staging for m <= 8 (GPSPCA_MFMA_HALF_X=0 turns it off, for tests and
// comparisons).
static bool mfma_half_x() {
    const char* e = std::getenv("GPSPCA_MFMA_HALF_X");
    return !(e && e[0] == '0');
}

static int corr_mfma_blocks_per_cu_query(int m, int stages);

// Resident workgroups per CU of the configuration (m bucket, stages): the
// occupancy query runs once per configuration; every plan (and every
// workspace-size query, which builds a plan per autotuner candidate) reuses it.
int corr_mfma_blocks_per_cu(int m, int stages) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cache;
    const std::pair<int, int> key(m <= 16 ? 16 : m <= 32 ? 32 : 64, stages);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int nb = corr_mfma_blocks_per_cu_query(m, stages);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = nb;
    return nb;
}

static int corr_mfma_blocks_per_cu_query(int m, int stages) {
    int nb = 0;
    hipError_t e;
    if (m <= 16 && stages == 8)  // wide chunks: 2 stages of 8 tiles
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<1, 2, 8>, 64, 0);
    else if (m <= 16 && stages == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<1, 4>, 64, 0);
    else if (m <= 16 && stages == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<1, 2>, 64, 0);
    else if (m <= 16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<1, 3>, 64, 0);
    else if (m <= 32 && stages == 8)  // wide chunks for two component groups
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<2, 2, 8>, 64, 0);
    else if (m <= 32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<2, 3>, 64, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_mfma<4, 2>, 64, 0);
    (void)hipGetLastError();
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_corr_mfma(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                            float* S, uint8_t* act, double* fpart, int* nnzpart, float* xpart,
                            const Ctrl* ctrl, hipStream_t st) {
    const dim3 grid(pl.corr_grid), block(64);
    BalArgs bal{xpart, pl.bal_q, pl.bal_rem, pl.nwave_part};
    const bool hx = pl.m <= 8 && mfma_half_x();
    if (pl.bal && hx && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 2, 8, true, true>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.bal && pl.m <= 16 && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 2, 8, false, true>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.bal && pl.m <= 32 && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<2, 2, 8, false, true>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (hx && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 2, 8, true>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 16 && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 2, 8>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 16 && pl.mfma_stages == 4)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 4>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 16 && pl.mfma_stages == 2)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 2>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 16)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<1, 3>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 32 && pl.mfma_stages == 8)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<2, 2, 8>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else if (pl.m <= 32)
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<2, 3>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    else
        GPSPCA_LAUNCH_TIMED((k_corr_mfma<4, 2>), grid, block, 0, st, pp, X, Xil, S, act, fpart, nnzpart, ctrl, bal);
    if (pl.bal) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (pl.m <= 16)
            hipLaunchKernelGGL(k_corr_bal_fix<1>, dim3(pl.bal_rem), dim3(64), 0, st, pp, bal,
                               pl.corr_grid, S, act, fpart, nnzpart, ctrl);
        else
            hipLaunchKernelGGL(k_corr_bal_fix<2>, dim3(pl.bal_rem), dim3(64), 0, st, pp, bal,
                               pl.corr_grid, S, act, fpart, nnzpart, ctrl);
    }
    return hipGetLastError();
}

}  // namespace gpspca
