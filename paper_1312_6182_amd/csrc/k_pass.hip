// Pass kernels of the GP-SPCA power iteration on gfx950: the only kernels that
// stream the data matrix A from HBM.
//
// One pass (Section 2, Table 1) computes, for every variable column a_i and
// component j:
//   y_ij = a_i^T x_j                                         (correlation)
//   l1: s_ij = sign(y_ij) [mu_j |y_ij| - gamma]_+ ,  f_j += [.]_+^2
//   l0: s_ij = mu_j y_ij if (mu_j y_ij)^2 > gamma,  f_j += (mu_j y_ij)^2 - gamma
//   g_j += mu_j s_ij a_i                                     (ascent direction)
//
// Kernels:
//  k_pass_m1   m = 1, single pass over A: each workgroup keeps x and its partial
//              of g in registers (rows distributed over threads), loads a batch
//              of columns, reduces the dot products across the workgroup, applies
//              the threshold and the axpy on the registers it already holds.
//  k_corr      block forms (m <= 8 per launch): one wavefront owns a contiguous
//              range of columns and computes B columns x M components of a_i^T X
//              per sweep over the rows (float4 loads, 64-value butterfly reduction),
//              thresholds in registers and writes S and a per-column activity flag.
//  k_backproj  block forms: G partials = sum over ACTIVE columns only of
//              a_i (mu * s_i)^T, so a sparse support costs a small fraction of a
//              second pass; workgroups own a (row block, column range) tile.
//              When enough of the pass's columns are active it instead runs
//              the dense form: every column of each range with an active
//              column, on the matrix cores (bpm_block), every component group
//              in one read of A.
//  k_colnorm   ||a_i|| in FP64 (default start).
#include "gpspca_internal.h"
#include "storage.h"

namespace gpspca {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

// Quad q (rows 4q..4q+3) of one column.  Full quads use one 16-byte load when
// the column is 16-byte aligned (VEC); the ragged last quad is masked.
template <bool VEC>
__device__ __forceinline__ f4 load_quad(const float* __restrict__ col, int q, int nqf, int p) {
    const int r = 4 * q;
    if (q < nqf) {
        if constexpr (VEC) {
            return __builtin_nontemporal_load(reinterpret_cast<const f4*>(col + r));
        } else {
            return f4{col[r], col[r + 1], col[r + 2], col[r + 3]};
        }
    }
    f4 v = zero4();
    if (r < p) v.x = col[r];
    if (r + 1 < p) v.y = col[r + 1];
    if (r + 2 < p) v.z = col[r + 2];
    if (r + 3 < p) v.w = col[r + 3];
    return v;
}

// One full quad (4 rows known to lie inside the column).
template <bool VEC>
__device__ __forceinline__ f4 load_full(const float* __restrict__ ptr) {
    if constexpr (VEC) {
        return __builtin_nontemporal_load(reinterpret_cast<const f4*>(ptr));
    } else {
        return f4{ptr[0], ptr[1], ptr[2], ptr[3]};
    }
}

__device__ __forceinline__ float dot4(f4 a, f4 b, float acc) {
    acc = __builtin_fmaf(a.x, b.x, acc);
    acc = __builtin_fmaf(a.y, b.y, acc);
    acc = __builtin_fmaf(a.z, b.z, acc);
    acc = __builtin_fmaf(a.w, b.w, acc);
    return acc;
}

// Threshold of one correlation (Table 1).  Returns true when the entry is in
// the support; s is the thresholded value and fv its objective term.
__device__ __forceinline__ bool threshold(bool l0, double mu, double gamma, float y, float& s,
                                          double& fv) {
    const double yd = (double)y;
    if (l0) {
        const double my = mu * yd;
        const double q = my * my - gamma;
        if (q > 0.0) {
            s = (float)my;
            fv = q;
            return true;
        }
    } else {
        const double t = mu * fabs(yd) - gamma;
        if (t > 0.0) {
            s = (float)(yd > 0.0 ? t : -t);
            fv = t * t;
            return true;
        }
    }
    s = 0.f;
    fv = 0.0;
    return false;
}

template <typename T>
__device__ __forceinline__ T wave_allreduce_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// k_pass_m1: fused single pass, m = 1.
//   T threads; thread t owns row quads t + T*k (k < KQ).  B columns per batch,
//   the next batch is loaded before the current one is reduced.
// ---------------------------------------------------------------------------
template <int T, int KQ, int B, bool VEC>
__global__ __launch_bounds__(T) void k_pass_m1(PassParams pp, const float* __restrict__ x,
                                               float* __restrict__ S, float* __restrict__ gpart,
                                               double* __restrict__ fpart,
                                               int* __restrict__ nnzpart,
                                               const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int NWV = T / 64;
    __shared__ float red[2][NWV][B];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int p = pp.p, nqf = p >> 2, nq = (p + 3) >> 2;
    const int64_t cb = pp.n * (int64_t)blockIdx.x / gridDim.x;
    const int64_t ce = pp.n * (int64_t)(blockIdx.x + 1) / gridDim.x;
    const bool l0 = pp.l0 != 0;
    const double gamma = pp.gam[0], mu = pp.mu[0];
    const float muf = pp.muf[0];

    f4 xr[KQ], g[KQ];
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
        const int q = t + T * k;
        xr[k] = (q < nq) ? *reinterpret_cast<const f4*>(x + 4 * q) : zero4();
        g[k] = zero4();
    }
    double f_acc = 0.0;
    int nnz_acc = 0;

    f4 a[B][KQ];
    // Loads of one batch: every full quad with one unconditional 16-byte load
    // (address clamped into the column, value zeroed past the last full quad),
    // then the ragged last quad (p % 4 rows) by its single owner thread.
    const int tail_t = nqf % T, tail_k = nqf / T;
    const bool has_tail = (p & 3) != 0;
    auto load_batch = [&](int64_t c0, f4(&dst)[B][KQ]) {
        const float* col[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t c = (c0 + b < ce) ? c0 + b : ce - 1;
            col[b] = pp.A + c * pp.lda;
        }
        if (nqf > 0) {
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < KQ; ++k) {
                    const int q = t + T * k;
                    const int qc = q < nqf ? q : nqf - 1;
                    dst[b][k] = load_full<VEC>(col[b] + 4 * qc);
                }
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < KQ; ++k)
                    if (t + T * k >= nqf) dst[b][k] = zero4();
        } else {
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < KQ; ++k) dst[b][k] = zero4();
        }
        if (has_tail && t == tail_t) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const f4 v = load_quad<false>(col[b], nqf, nqf, p);
#pragma unroll
                for (int k = 0; k < KQ; ++k)
                    if (k == tail_k) dst[b][k] = v;
            }
        }
    };
    if (cb < ce) load_batch(cb, a);

    int it = 0;
    for (int64_t c0 = cb; c0 < ce; c0 += B, ++it) {
        float d[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < KQ; ++k) acc = dot4(a[b][k], xr[k], acc);
            d[b] = acc;
        }
        const bool more = c0 + B < ce;
        f4 an[B][KQ];
        if (more) load_batch(c0 + B, an);
#pragma unroll
        for (int b = 0; b < B; ++b) d[b] = wave_allreduce_sum(d[b]);
        if (lane == 0) {
#pragma unroll
            for (int b = 0; b < B; ++b) red[it & 1][wv][b] = d[b];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            float y = 0.f;
#pragma unroll
            for (int w = 0; w < NWV; ++w) y += red[it & 1][w][b];
            if (c0 + b < ce) {
                float s;
                double fv;
                const bool act = threshold(l0, mu, gamma, y, s, fv);
                if (act) {
                    const float wgt = muf * s;
#pragma unroll
                    for (int k = 0; k < KQ; ++k) {
                        g[k].x = __builtin_fmaf(wgt, a[b][k].x, g[k].x);
                        g[k].y = __builtin_fmaf(wgt, a[b][k].y, g[k].y);
                        g[k].z = __builtin_fmaf(wgt, a[b][k].z, g[k].z);
                        g[k].w = __builtin_fmaf(wgt, a[b][k].w, g[k].w);
                    }
                    if (t == 0) {
                        f_acc += fv;
                        nnz_acc += 1;
                    }
                }
                if (t == 0) S[c0 + b] = s;
            }
        }
        if (more) {
#pragma unroll
            for (int b = 0; b < B; ++b)
#pragma unroll
                for (int k = 0; k < KQ; ++k) a[b][k] = an[b][k];
        }
    }
    float* gp = gpart + (size_t)blockIdx.x * pp.ldx;
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
        const int q = t + T * k;
        if (q < nq) *reinterpret_cast<f4*>(gp + 4 * q) = g[k];
    }
    if (t == 0) {
        fpart[blockIdx.x] = f_acc;
        nnzpart[blockIdx.x] = nnz_acc;
    }
}

// ---------------------------------------------------------------------------
// k_corr: correlation + threshold for the block forms.
//   M components (padded, m_g <= M real ones starting at j0), B columns per
//   sweep, V = B*M = 64 accumulators per lane reduced by a butterfly so that lane
//   l ends with value (b, j) = (l / M, l % M) (V = 64) or shared by 64/V lanes.
// ---------------------------------------------------------------------------
template <int O, int S, int V>
__device__ __forceinline__ void butterfly(float (&v)[V], int lane) {
    if constexpr (O >= 1) {
        if constexpr (S > 1) {
            constexpr int H = S / 2;
            const bool up = (lane & O) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const float send = up ? v[i] : v[i + H];
                const float keep = up ? v[i + H] : v[i];
                v[i] = keep + __shfl_xor(send, O, 64);
            }
            butterfly<O / 2, H, V>(v, lane);
        } else {
            v[0] += __shfl_xor(v[0], O, 64);
            butterfly<O / 2, 1, V>(v, lane);
        }
    }
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <int M, int B, bool VEC>
__global__ __launch_bounds__(256) void k_corr(PassParams pp, int j0, const float* __restrict__ X,
                                              float* __restrict__ S, uint8_t* __restrict__ act,
                                              double* __restrict__ fpart,
                                              int* __restrict__ nnzpart,
                                              const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int V = B * M;
    static_assert(V <= 64 && (V & (V - 1)) == 0, "B*M must be a power of two <= 64");
    constexpr int SHIFT = 6 - ilog2c(V);
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    // columns visited: all n, or the frozen-support list
    const int64_t nv = pp.list ? (int64_t)*pp.nlist : pp.n;
    const int64_t cb = nv * wave / nw, ce = nv * (wave + 1) / nw;
    const int p = pp.p, nqf = p >> 2;
    const int m = pp.m;
    const int mg = (m - j0 < M) ? m - j0 : M;  // real components in this launch
    const bool l0 = pp.l0 != 0;

    const int vidx = lane >> SHIFT;
    const int ob = vidx / M, oj = vidx % M;
    const bool rep = (lane & ((1 << SHIFT) - 1)) == 0;
    const double muj = (oj < mg) ? pp.mu[j0 + oj] : 1.0;
    uint64_t grpmask = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) grpmask |= 1ull << (j << SHIFT);

    const float* Xg = X + (size_t)j0 * pp.ldx;
    double f_acc = 0.0;
    int nnz_acc = 0;

    for (int64_t c0 = cb; c0 < ce; c0 += B) {
        const float* colp[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int64_t v = (c0 + b < ce) ? c0 + b : ce - 1;
            const int64_t c = pp.list ? (int64_t)pp.list[v] : v;
            colp[b] = pp.A + c * pp.lda;
        }
        float acc[V];
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = 0.f;
        // full row quads: unconditional 16-byte loads (X is padded with zero
        // components up to a multiple of M, so no component guard is needed)
        for (int q = lane; q < nqf; q += 64) {
            f4 xv[M];
#pragma unroll
            for (int j = 0; j < M; ++j)
                xv[j] = *reinterpret_cast<const f4*>(Xg + (size_t)j * pp.ldx + 4 * q);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const f4 a = load_full<VEC>(colp[b] + 4 * q);
#pragma unroll
                for (int j = 0; j < M; ++j) acc[b * M + j] = dot4(a, xv[j], acc[b * M + j]);
            }
        }
        // ragged tail rows 4*nqf .. p-1 (at most 3), one lane per row
        if (lane < p - 4 * nqf) {
            const int r = 4 * nqf + lane;
            float xs[M];
#pragma unroll
            for (int j = 0; j < M; ++j) xs[j] = Xg[(size_t)j * pp.ldx + r];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const float a = colp[b][r];
#pragma unroll
                for (int j = 0; j < M; ++j) acc[b * M + j] = __builtin_fmaf(a, xs[j], acc[b * M + j]);
            }
        }
        butterfly<32, V, V>(acc, lane);
        const float y = acc[0];
        const bool valid = rep && (c0 + ob < ce) && (oj < mg);
        const int64_t col = !valid ? 0 : pp.list ? (int64_t)pp.list[c0 + ob] : c0 + ob;
        bool active = false;
        if (valid) {
            float s;
            double fv;
            active = threshold(l0, muj, pp.gam[j0 + oj], y, s, fv);
            if (pp.mask && !((pp.mask[(int64_t)(j0 + oj) * pp.mask_words + (col >> 5)] >> (col & 31)) & 1u)) {
                active = false;
                s = 0.f;
            }
            S[col * m + j0 + oj] = s;
            if (active) {
                f_acc += fv;
                nnz_acc += 1;
            }
        }
        const uint64_t bal = __ballot(active);
        if (valid && oj == 0) {
            const bool any = (bal & (grpmask << ((ob * M) << SHIFT))) != 0;
            if (j0 == 0) act[col] = any ? 1 : 0;
            else if (any) act[col] = 1;
        }
    }
    // Per-component totals over the lanes that share oj (fixed xor order).
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        if (o >= (1 << SHIFT) && o < (M << SHIFT)) continue;
        f_acc += __shfl_xor(f_acc, o, 64);
        nnz_acc += __shfl_xor(nnz_acc, o, 64);
    }
    if (ob == 0 && rep && oj < mg) {
        fpart[(int64_t)(j0 + oj) * nw + wave] = f_acc;
        nnzpart[(int64_t)(j0 + oj) * nw + wave] = nnz_acc;
    }
}


// ---------------------------------------------------------------------------
// k_corr_vx: correlation + threshold for m <= 8 with X held in registers.
//   T threads; thread t owns row quads t + T*k (k < KQ) and keeps X on those
//   rows (KQ x M float4) for the whole pass.  The workgroup walks its
//   contiguous column range one column at a time: every wave-load is 1 KB of
//   one column (contiguous, like a flat stream), the next column is loaded
//   before the current one is reduced, the M partial dots are reduced by a
//   transposed butterfly (lane groups of 64/M keep one component) and across
//   the waves through LDS (one barrier per column), and thread j < M applies
//   the threshold of component j.
// ---------------------------------------------------------------------------
template <int T, int KQ, int M, bool VEC>
__global__ __launch_bounds__(T) void k_corr_vx(PassParams pp, const float* __restrict__ X,
                                               float* __restrict__ S, uint8_t* __restrict__ act,
                                               double* __restrict__ fpart,
                                               int* __restrict__ nnzpart,
                                               const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int NWV = T / 64;
    constexpr int SHIFT = 6 - ilog2c(M);  // lanes per component after the butterfly
    __shared__ float red[2][NWV][M];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int p = pp.p, nqf = p >> 2, m = pp.m, ldx = pp.ldx;
    const int64_t cb = pp.n * (int64_t)blockIdx.x / gridDim.x;
    const int64_t ce = pp.n * (int64_t)(blockIdx.x + 1) / gridDim.x;
    int nact_t = 0;   // active columns (thread 0 writes the flags)
    const bool l0 = pp.l0 != 0;
    const int tail_t = nqf % T, tail_k = nqf / T;
    const bool has_tail = (p & 3) != 0;

    f4 xr[KQ][M];
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
        const int q = t + T * k;
#pragma unroll
        for (int j = 0; j < M; ++j)
            xr[k][j] = (4 * q < ldx) ? *reinterpret_cast<const f4*>(X + (size_t)j * ldx + 4 * q)
                                     : zero4();
    }
    // component handled by this thread in the threshold step (t < M)
    const int mj = t < M ? t : 0;
    const double muj = pp.mu[mj], gamj = pp.gam[mj];
    double f_acc = 0.0;
    int nnz_acc = 0;

    auto load_col = [&](int64_t c, f4(&dst)[KQ]) {
        const float* col = pp.A + c * pp.lda;
        if (nqf > 0) {
#pragma unroll
            for (int k = 0; k < KQ; ++k) {
                const int q = t + T * k;
                const int qc = q < nqf ? q : nqf - 1;
                dst[k] = load_full<VEC>(col + 4 * qc);
            }
#pragma unroll
            for (int k = 0; k < KQ; ++k)
                if (t + T * k >= nqf) dst[k] = zero4();
        } else {
#pragma unroll
            for (int k = 0; k < KQ; ++k) dst[k] = zero4();
        }
        if (has_tail && t == tail_t) {
            const f4 v = load_quad<false>(col, nqf, nqf, p);
#pragma unroll
            for (int k = 0; k < KQ; ++k)
                if (k == tail_k) dst[k] = v;
        }
    };

    f4 a[KQ];
    if (cb < ce) load_col(cb, a);
    int it = 0;
    for (int64_t c = cb; c < ce; ++c, ++it) {
        float d[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < KQ; ++k) acc = dot4(a[k], xr[k][j], acc);
            d[j] = acc;
        }
        f4 an[KQ];
        const bool more = c + 1 < ce;
        if (more) load_col(c + 1, an);
        butterfly<32, M, M>(d, lane);
        if ((lane & ((1 << SHIFT) - 1)) == 0) red[it & 1][wv][lane >> SHIFT] = d[0];
        __syncthreads();
        bool active = false;
        if (t < M) {
            float y = 0.f;
#pragma unroll
            for (int w = 0; w < NWV; ++w) y += red[it & 1][w][t];
            if (t < m) {
                float sv;
                double fv;
                active = threshold(l0, muj, gamj, y, sv, fv);
                S[c * m + t] = sv;
                if (active) {
                    f_acc += fv;
                    nnz_acc += 1;
                }
            }
        }
        const uint64_t bal = __ballot(active);
        if (t == 0) {
            const int fl = (bal & ((1ull << M) - 1ull)) ? 1 : 0;
            act[c] = fl;
            nact_t += fl;
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < KQ; ++k) a[k] = an[k];
        }
    }
    if (t < m) {
        fpart[(int64_t)t * gridDim.x + blockIdx.x] = f_acc;
        nnzpart[(int64_t)t * gridDim.x + blockIdx.x] = nnz_acc;
    }
    if (t == 0 && nact_t > 0 && pp.nact) atomicAdd(pp.nact, nact_t);
}

// ---------------------------------------------------------------------------
// Dense or sparse back-projection.  The pass is back-projected densely iff at
// least thr/1024 of all n columns are active (the correlation kernels count
// them into *pp.nact): then every column range with an active column is taken
// by the dense form of k_backproj, and the others (nothing to add) by its
// sparse form.  One decision for the whole pass: a dense range costs a full
// read of its columns by a few waves, so a pass with only some dense ranges
// would wait on them.  thr > kBpThrMax: never.
// ---------------------------------------------------------------------------
constexpr int kBpThrMax = 1024;

__device__ __forceinline__ bool pass_is_dense(const PassParams& pp, int thr) {
    if (thr > kBpThrMax || !pp.nact) return false;
    const int64_t na = *pp.nact;
    return na > 0 && na * kBpThrMax >= (int64_t)thr * pp.n;
}

// This thread's share of the active columns of [cb, ce) (flags are 0 or 1),
// read as aligned 32-bit words of the flag array, whose allocation is padded
// to 256 bytes; bytes outside the range are masked off.
__device__ __forceinline__ int count_active(const uint8_t* __restrict__ act, int64_t cb,
                                            int64_t ce, int tid, int nthreads) {
    const uint32_t* aw = reinterpret_cast<const uint32_t*>(act);
    const int64_t w0 = cb >> 2, w1 = (ce + 3) >> 2;
    int c = 0;
#pragma unroll 4
    for (int64_t w = w0 + tid; w < w1; w += nthreads) {
        uint32_t v = aw[w];
        const int64_t lo = cb - 4 * w, hi = 4 * w + 4 - ce;
        if (lo > 0) v &= 0xFFFFFFFFu << (8 * lo);
        if (hi > 0) v &= 0xFFFFFFFFu >> (8 * hi);
        c += __popc(v);
    }
    return c;
}


// ---------------------------------------------------------------------------
// bpm_block: dense G partial of column range cr = A[:, cb:ce] W[cb:ce, :],
// W_ij = mu_j s_ij scale_i, over every column of the range, on the matrix
// cores (v_mfma_f32_16x16x4_f32: 16 rows x 16 components, contraction over 4
// columns).
//   grid (row blocks of 64 RL rows, four per workgroup; column ranges); every
//   component group (G of 16) in the same read of A.
//   Lane (li, lk) = (l % 16, l / 16) loads quad q0 + li + 16 r (r < RL) of
//   column c + lk; that one load feeds the four tiles (r, e), whose operand row
//   li is data row 4 (q0 + li + 16 r) + e, against the weight of column
//   c + lk, component 16 g + li.  Accumulator register v of tile (r, e) then
//   holds data row 4 (q0 + 16 r + 4 lk + v) + e, so each lane stores whole
//   quads.
//   Steps of 4 columns are software-pipelined D deep with compile-time buffer
//   indices.  Columns past the range are clamped and weighted 0; quads past
//   the last full one are clamped and replaced by the ragged rows or zeros
//   (TAIL, the last row block only), so no load is conditional.
// ---------------------------------------------------------------------------
// Raw (undecoded) storage of one full quad, and its decoding; the tail quad
// is kept as four raw elements.
template <int ST> struct QuadRaw { using T = f4; };
template <> struct QuadRaw<kStBF16> { using T = uint2; };
template <> struct QuadRaw<kStF8> { using T = uint32_t; };

template <int ST>
__device__ __forceinline__ typename QuadRaw<ST>::T load_quad_raw(const void* colv, int q) {
    using T = typename QuadRaw<ST>::T;
    if constexpr (ST == kStF32)
        return __builtin_nontemporal_load(reinterpret_cast<const f4*>(static_cast<const float*>(colv) + 4 * q));
    else if constexpr (ST == kStBF16)
        return *reinterpret_cast<const T*>(static_cast<const uint16_t*>(colv) + 4 * q);
    else
        return *reinterpret_cast<const T*>(static_cast<const uint8_t*>(colv) + 4 * q);
}

// Raw full quad for the support-restricted back-projection: FP32 columns
// whose leading dimension is not a multiple of 4 are read element-wise.
template <int ST, bool VEC>
__device__ __forceinline__ typename QuadRaw<ST>::T load_raw_sp(const void* colv, int q) {
    if constexpr (ST == kStF32 && !VEC) {
        const float* c = static_cast<const float*>(colv) + 4 * q;
        return f4{c[0], c[1], c[2], c[3]};
    } else {
        return load_quad_raw<ST>(colv, q);
    }
}

template <int ST>
__device__ __forceinline__ f4 decode_quad(typename QuadRaw<ST>::T w) {
    if constexpr (ST == kStF32) {
        return w;
    } else if constexpr (ST == kStBF16) {
        return f4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                  __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u)};
    } else {
        const qf2 lo = e4m3_pair(w, false), hi = e4m3_pair(w, true);
        return f4{lo.x, lo.y, hi.x, hi.y};
    }
}

template <int ST>
__device__ __forceinline__ uint32_t load_elem_raw(const void* colv, int r) {
    if constexpr (ST == kStF32) return __float_as_uint(static_cast<const float*>(colv)[r]);
    else if constexpr (ST == kStBF16) return static_cast<const uint16_t*>(colv)[r];
    else return static_cast<const uint8_t*>(colv)[r];
}

template <int ST>
__device__ __forceinline__ float decode_elem(uint32_t w) {
    if constexpr (ST == kStF32) return __uint_as_float(w);
    else if constexpr (ST == kStBF16) return bf16_value(w);
    else return e4m3_value(w);
}

template <int RL, int G, int D, bool TAIL, int ST>
__device__ __forceinline__ void bpm_block(const PassParams& pp, int64_t cb, int64_t ce, int q0,
                                          const float* __restrict__ S,
                                          float* __restrict__ gp) {
    using RawT = typename QuadRaw<ST>::T;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m, nqf = p >> 2, nq = (p + 3) >> 2;
    float mul[G];
    int comp[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int j = 16 * g + li;
        mul[g] = (j < m) ? pp.muf[j] : 0.f;
        comp[g] = (j < m) ? j : m - 1;
    }
    int qa[RL];
    bool full[RL], tailq[RL];
#pragma unroll
    for (int r = 0; r < RL; ++r) {
        const int q = q0 + li + 16 * r;
        qa[r] = (q < nqf) ? q : nqf - 1;
        full[r] = q < nqf;
        tailq[r] = q == nqf;
    }
    int trow[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) trow[e] = (4 * nqf + e < p) ? 4 * nqf + e : p - 1;

    // loads only fill registers; decoding and weighting happen where the
    // operands are consumed, so no wait sits between a load and its prefetch slot
    struct Buf {
        RawT a[RL];
        uint32_t t[TAIL ? 4 : 1];
        float s[G];
        float sc;
    };
    auto load = [&](int64_t step, Buf& b) {
        const int64_t c = cb + 4 * step + lk;
        const int64_t cc = (c < ce) ? c : ce - 1;
        const void* colv = column_ptr<ST>(pp, cc);
#pragma unroll
        for (int r = 0; r < RL; ++r) b.a[r] = load_quad_raw<ST>(colv, qa[r]);
        if constexpr (TAIL) {
#pragma unroll
            for (int e = 0; e < 4; ++e) b.t[e] = load_elem_raw<ST>(colv, trow[e]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) b.s[g] = S[cc * m + comp[g]];
        if constexpr (ST != kStF32) b.sc = column_scale(pp, cc);
    };
    f4 acc[RL][4][G];
#pragma unroll
    for (int r = 0; r < RL; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int g = 0; g < G; ++g) acc[r][e][g] = zero4();

    const int64_t nstep = (ce - cb + 3) / 4;
    Buf buf[D];
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, buf[d]);
    __builtin_amdgcn_sched_barrier(0);
    // steps past the last one are clamped loads with zero weights
    for (int64_t s0 = 0; s0 < nstep; s0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const Buf& b = buf[d];
            const float valid = (cb + 4 * (s0 + d) + lk < ce) ? 1.f : 0.f;
            float w[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                float wv = mul[g] * b.s[g];
                if constexpr (ST != kStF32) wv *= b.sc;
                w[g] = wv * valid;
            }
            f4 a[RL];
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                a[r] = decode_quad<ST>(b.a[r]);
                if constexpr (TAIL) {
                    f4 rag;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rag[e] = (4 * nqf + e < p) ? decode_elem<ST>(b.t[e]) : 0.f;
                    a[r] = full[r] ? a[r] : (tailq[r] ? rag : zero4());
                }
            }
#pragma unroll
            for (int r = 0; r < RL; ++r)
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        acc[r][e][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            a[r][e], w[g], acc[r][e][g], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            load(s0 + d + D, buf[d]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

#pragma unroll
    for (int r = 0; r < RL; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int qw = q0 + 16 * r + 4 * lk + v;
            if (qw < nq) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int j = 16 * g + li;
                    if (j < m)
                        *reinterpret_cast<f4*>(gp + (size_t)j * pp.ldx + 4 * qw) =
                            f4{acc[r][0][g][v], acc[r][1][g][v], acc[r][2][g][v], acc[r][3][g][v]};
                }
            }
        }
}

// ---------------------------------------------------------------------------
// k_backproj: G partial of column range cr.
//   grid (row blocks, column ranges); 256 threads.
//   Sparse pass: thread t owns quads qbase + t + 256 k (k < KQ2) of the row
//   block and adds the active columns, U per step, for components j0 .. j0+M-1.
//   Dense pass, G = 1 (m <= 16): the workgroup's four waves take row blocks of
//   256 rows in turn and run bpm_block over every column of a range that has
//   an active column.  One launch serves both, so a sparse pass pays no launch
//   for the dense code.  (m > 16: k_backproj_dense, below.)
// ---------------------------------------------------------------------------
template <int M, int KQ2, bool VEC, int ST, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_backproj(
                                                  PassParams pp, int j0b,
                                                  const float* __restrict__ S,
                                                  const uint8_t* __restrict__ act,
                                                  float* __restrict__ gpart,
                                                  int* __restrict__ touched, int ncr, int thr,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int U = 4;
    __shared__ int list[256];
    __shared__ int wcount[4];
    // component group of this workgroup: launches cover several groups of 16
    // components through the grid's z dimension
    const int j0 = j0b + 16 * (int)blockIdx.z;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int p = pp.p, nqf = p >> 2, nq = (p + 3) >> 2, m = pp.m;
    const int mg = (m - j0 < M) ? m - j0 : M;
    const int qbase = blockIdx.x * 256 * KQ2;
    const int cr = blockIdx.y;
    const int64_t cb = pp.n * cr / ncr, ce = pp.n * (cr + 1) / ncr;
    if (pass_is_dense(pp, thr)) {
        // dense pass: ranges with an active column are read in full
        int c = count_active(act, cb, ce, t, 256);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) wcount[wv] = c;
        __syncthreads();
        const int64_t total = (int64_t)wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (total > 0) {
            if constexpr (G > 0) {
                if (j0 == 0) {
                    constexpr int RL = G <= 2 ? 4 : 2;
                    const int nrb = (nq + 16 * RL - 1) / (16 * RL);
                    float* gp = gpart + (size_t)cr * m * pp.ldx;
                    for (int rb = blockIdx.x * 4 + wv; rb < nrb; rb += 4 * gridDim.x) {
                        const int q0 = rb * 16 * RL;
                        if (q0 + 16 * RL > nqf)
                            bpm_block<RL, G, 3, true, ST>(pp, cb, ce, q0, S, gp);
                        else
                            bpm_block<RL, G, 3, false, ST>(pp, cb, ce, q0, S, gp);
                    }
                    if (blockIdx.x == 0 && t == 0) touched[cr] = 1;
                }
            }
            return;
        }
        __syncthreads();
    }

    f4 g[KQ2][M];
#pragma unroll
    for (int k = 0; k < KQ2; ++k)
#pragma unroll
        for (int j = 0; j < M; ++j) g[k][j] = zero4();
    bool any = false;
    // mu of the group's components, 0 past the group (those weights vanish)
    float mw[M];
#pragma unroll
    for (int j = 0; j < M; ++j) mw[j] = (j < mg) ? pp.muf[j0 + j] : 0.f;
    // this thread's quads (the same in every column): full ones, the ragged
    // tail quad of rows 4 nqf .. p - 1, or none
    using RawT = typename QuadRaw<ST>::T;
    const bool ragged = (p & 3) != 0;
    int qa[KQ2];
    bool full[KQ2], tq[KQ2];
#pragma unroll
    for (int k = 0; k < KQ2; ++k) {
        const int q = qbase + t + 256 * k;
        qa[k] = (q < nqf) ? q : (nqf > 0 ? nqf - 1 : 0);
        full[k] = q < nqf;
        tq[k] = ragged && q == nqf;
    }
    int trow[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) trow[x] = (4 * nqf + x < p) ? 4 * nqf + x : p - 1;

    for (int64_t base = cb; base < ce; base += 256) {
        const int64_t i = base + t;
        const bool fl = (i < ce) && act[i] != 0;
        const uint64_t bal = __ballot(fl);
        if (lane == 0) wcount[wv] = __popcll(bal);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wv; ++w) off += wcount[w];
        const int total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        if (fl) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = t;
        __syncthreads();
        for (int e = 0; e < total; e += U) {
            f4 a[U][KQ2];
            float w[U][M];
            // Every load below is unconditional and only fills registers
            // (components past the group re-read its last one with weight 0;
            // quads past the last full one re-read it and are replaced by the
            // ragged rows or zeros at decoding), so the loads of the U columns
            // are issued together instead of each behind its own branch and wait.
            RawT ra[U][KQ2];
            uint32_t rt[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int li = (e + u < total) ? list[e + u] : list[e];
                const int64_t col = base + li;
                const void* colv = column_ptr<ST>(pp, col);
                const float sc = (ST == kStF32) ? 1.0f : column_scale(pp, col);
#pragma unroll
                for (int j = 0; j < M; ++j)
                    w[u][j] = mw[j] * S[col * m + j0 + (j < mg ? j : mg - 1)] * sc;
                if (nqf > 0) {
#pragma unroll
                    for (int k = 0; k < KQ2; ++k) ra[u][k] = load_raw_sp<ST, VEC>(colv, qa[k]);
                }
                if (ragged) {
#pragma unroll
                    for (int x = 0; x < 4; ++x) rt[u][x] = load_elem_raw<ST>(colv, trow[x]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < KQ2; ++k) {
                    f4 v = zero4();
                    if (nqf > 0) v = decode_quad<ST>(ra[u][k]);
                    if (ragged) {
                        f4 rag;
#pragma unroll
                        for (int x = 0; x < 4; ++x)
                            rag[x] = (4 * nqf + x < p) ? decode_elem<ST>(rt[u][x]) : 0.f;
                        v = tq[k] ? rag : v;
                    }
                    a[u][k] = (full[k] || tq[k]) ? v : zero4();
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e + u < total) {
#pragma unroll
                    for (int k = 0; k < KQ2; ++k)
#pragma unroll
                        for (int j = 0; j < M; ++j) {
                            g[k][j].x = __builtin_fmaf(w[u][j], a[u][k].x, g[k][j].x);
                            g[k][j].y = __builtin_fmaf(w[u][j], a[u][k].y, g[k][j].y);
                            g[k][j].z = __builtin_fmaf(w[u][j], a[u][k].z, g[k][j].z);
                            g[k][j].w = __builtin_fmaf(w[u][j], a[u][k].w, g[k][j].w);
                        }
                }
            }
        }
        any = any || total > 0;
        __syncthreads();
    }
    if (any) {
        float* gp = gpart + (size_t)cr * m * pp.ldx;
#pragma unroll
        for (int k = 0; k < KQ2; ++k) {
            const int q = qbase + t + 256 * k;
            if (q < nq) {
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j < mg)
                        *reinterpret_cast<f4*>(gp + (size_t)(j0 + j) * pp.ldx + 4 * q) = g[k][j];
            }
        }
    }
    if (t == 0 && blockIdx.x == 0 && j0 == 0) touched[cr] = any ? 1 : 0;
}

// ---------------------------------------------------------------------------
// k_colnorm: ||a_i||_2 with FP64 accumulation; one wavefront per column range,
// four columns in flight.
// ---------------------------------------------------------------------------
template <bool VEC, int ST>
__global__ __launch_bounds__(256) void k_colnorm(PassParams pp, double* __restrict__ norms) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t cb = pp.n * wave / nw, ce = pp.n * (wave + 1) / nw;
    const int p = pp.p, nqf = p >> 2, nq = (p + 3) >> 2;
    constexpr int C = 4;
    for (int64_t c0 = cb; c0 < ce; c0 += C) {
        double s[C];
        const void* colp[C];
#pragma unroll
        for (int b = 0; b < C; ++b) {
            s[b] = 0.0;
            const int64_t c = (c0 + b < ce) ? c0 + b : ce - 1;
            colp[b] = column_ptr<ST>(pp, c);
        }
        for (int q = lane; q < nq; q += 64) {
#pragma unroll
            for (int b = 0; b < C; ++b) {
                f4 a;
                if constexpr (ST == kStF32)
                    a = load_quad<VEC>(static_cast<const float*>(colp[b]), q, nqf, p);
                else
                    a = load_quad_st<ST>(colp[b], q, nqf, p);
                s[b] += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z +
                        (double)a.w * a.w;
            }
        }
#pragma unroll
        for (int b = 0; b < C; ++b) {
            const double tot = wave_allreduce_sum(s[b]);
            if (lane == 0 && c0 + b < ce) {
                const double sc = (ST == kStF32) ? 1.0 : (double)column_scale(pp, c0 + b);
                norms[c0 + b] = sc * sqrt(tot);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int T, int KQ, bool VEC>
static hipError_t launch_m1_t(const Plan& pl, const PassParams& pp, const float* x, float* S,
                              float* gpart, double* fpart, int* nnzpart, const Ctrl* ctrl,
                              hipStream_t st) {
    GPSPCA_LAUNCH_TIMED((k_pass_m1<T, KQ, 2, VEC>), dim3(pl.m1_grid), dim3(T), 0, st, pp, x, S,
                       gpart, fpart, nnzpart, ctrl);
    return hipGetLastError();
}

template <int T, bool VEC>
static hipError_t launch_m1_kq(const Plan& pl, const PassParams& pp, const float* x, float* S,
                               float* gpart, double* fpart, int* nnzpart, const Ctrl* ctrl,
                               hipStream_t st) {
    switch (pl.m1_kq) {
        case 1: return launch_m1_t<T, 1, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 2: return launch_m1_t<T, 2, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 3: return launch_m1_t<T, 3, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 4: return launch_m1_t<T, 4, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 5: return launch_m1_t<T, 5, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        default: return hipErrorInvalidValue;
    }
}

template <bool VEC>
static hipError_t launch_m1_v(const Plan& pl, const PassParams& pp, const float* x, float* S,
                              float* gpart, double* fpart, int* nnzpart, const Ctrl* ctrl,
                              hipStream_t st) {
    switch (pl.m1_threads) {
        case 64: return launch_m1_kq<64, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 256: return launch_m1_kq<256, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 512: return launch_m1_kq<512, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        case 1024: return launch_m1_kq<1024, VEC>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pass_m1(const Plan& pl, const PassParams& pp, const float* x, float* S,
                          float* gpart, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    return pl.vec4 ? launch_m1_v<true>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st)
                   : launch_m1_v<false>(pl, pp, x, S, gpart, fpart, nnzpart, ctrl, st);
}

template <int M, int B, bool VEC>
static hipError_t launch_corr_t(const Plan& pl, const PassParams& pp, int j0, const float* X,
                                float* S, uint8_t* act, double* fpart, int* nnzpart,
                                const Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL((k_corr<M, B, VEC>), dim3(pl.corr_grid), dim3(256), 0, st, pp, j0, X, S,
                       act, fpart, nnzpart, ctrl);
    return hipGetLastError();
}

template <bool VEC>
static hipError_t launch_corr_v(const Plan& pl, const PassParams& pp, int j0, const float* X,
                                float* S, uint8_t* act, double* fpart, int* nnzpart,
                                const Ctrl* ctrl, hipStream_t st) {
    switch (pl.corr_M) {
        case 1: return launch_corr_t<1, 16, VEC>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st);
        case 2: return launch_corr_t<2, 16, VEC>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st);
        case 4: return launch_corr_t<4, 16, VEC>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st);
        case 8: return launch_corr_t<8, 8, VEC>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corr(const Plan& pl, const PassParams& pp, const float* X, float* S,
                       uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                       hipStream_t st) {
    for (int j0 = 0; j0 < pl.m; j0 += pl.corr_M) {
        hipError_t e = pl.vec4 ? launch_corr_v<true>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st)
                               : launch_corr_v<false>(pl, pp, j0, X, S, act, fpart, nnzpart, ctrl, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


template <int T, int KQ, int M>
static hipError_t launch_vx_t(const Plan& pl, const PassParams& pp, const float* X, float* S,
                              uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                              hipStream_t st) {
    GPSPCA_LAUNCH_TIMED((k_corr_vx<T, KQ, M, true>), dim3(pl.corr_grid), dim3(T), 0, st, pp, X, S,
                       act, fpart, nnzpart, ctrl);
    return hipGetLastError();
}

template <int T, int M>
static hipError_t launch_vx_kq(const Plan& pl, const PassParams& pp, const float* X, float* S,
                               uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                               hipStream_t st) {
    switch (pl.vx_kq) {
        case 1: return launch_vx_t<T, 1, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 2: return launch_vx_t<T, 2, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 3: return launch_vx_t<T, 3, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 4: return launch_vx_t<T, 4, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 5: return launch_vx_t<T, 5, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        default: return hipErrorInvalidValue;
    }
}

template <int M>
static hipError_t launch_vx_m(const Plan& pl, const PassParams& pp, const float* X, float* S,
                              uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                              hipStream_t st) {
    return pl.vx_threads == 256 ? launch_vx_kq<256, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st)
                                : launch_vx_kq<512, M>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
}

hipError_t launch_corr_vx(const Plan& pl, const PassParams& pp, const float* X, float* S,
                          uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    switch (pl.corr_M) {
        case 2: return launch_vx_m<2>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 4: return launch_vx_m<4>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        case 8: return launch_vx_m<8>(pl, pp, X, S, act, fpart, nnzpart, ctrl, st);
        default: return hipErrorInvalidValue;
    }
}

// Dense pass with more than one component group (m > 16): a launch of its
// own (merged into k_backproj, the dense code would spill registers); four
// waves per workgroup, each with its own row block.
template <int RL, int G, int ST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_backproj_dense(
    PassParams pp, const float* __restrict__ S, const uint8_t* __restrict__ act,
    float* __restrict__ gpart, int* __restrict__ touched, int ncr, int thr,
    const Ctrl* __restrict__ ctrl) {
    if (ctrl->done || !pass_is_dense(pp, thr)) return;
    const int lane = threadIdx.x & 63;
    const int q0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 * RL;
    if (q0 >= ((pp.p + 3) >> 2)) return;   // past the last row block (whole wave)
    const int cr = blockIdx.y;
    const int64_t cb = pp.n * cr / ncr, ce = pp.n * (cr + 1) / ncr;
    int c = count_active(act, cb, ce, lane, 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (c == 0) return;
    float* gp = gpart + (size_t)cr * pp.m * pp.ldx;
    if (q0 + 16 * RL > (pp.p >> 2))
        bpm_block<RL, G, 3, true, ST>(pp, cb, ce, q0, S, gp);
    else
        bpm_block<RL, G, 3, false, ST>(pp, cb, ce, q0, S, gp);
    if (blockIdx.x == 0 && threadIdx.x == 0) touched[cr] = 1;
}

template <int ST>
static hipError_t launch_bp_dense(const Plan& pl, const PassParams& pp, const float* S,
                                  const uint8_t* act, float* gpart, int* touched,
                                  const Ctrl* ctrl, hipStream_t st) {
    const int nq = (int)((pl.p + 3) / 4);
    const int qb = pl.m <= 32 ? 64 : 32;   // quads per row block: 16 RL
    const int nrb = (nq + qb - 1) / qb;
    const dim3 grid((unsigned)((nrb + 3) / 4), pl.bp_cr), block(256);
    if (pl.m <= 32)
        hipLaunchKernelGGL((k_backproj_dense<4, 2, ST>), grid, block, 0, st, pp, S, act, gpart,
                           touched, pl.bp_cr, pl.bp_thr, ctrl);
    else
        hipLaunchKernelGGL((k_backproj_dense<2, 4, ST>), grid, block, 0, st, pp, S, act, gpart,
                           touched, pl.bp_cr, pl.bp_thr, ctrl);
    return hipGetLastError();
}

// ng: component groups of 16 from j0 on, one per grid z index.
template <int M, bool VEC, int ST, int G>
static hipError_t launch_bp_t(const Plan& pl, const PassParams& pp, int j0, const float* S,
                              const uint8_t* act, float* gpart, int* touched, const Ctrl* ctrl,
                              hipStream_t st, int ng = 1) {
    hipLaunchKernelGGL((k_backproj<M, 2, VEC, ST, G>), dim3(pl.bp_rb, pl.bp_cr, ng), dim3(256), 0,
                       st, pp, j0, S, act, gpart, touched, pl.bp_cr, pl.bp_thr, ctrl);
    return hipGetLastError();
}

// With m <= 16 the launch carries the dense code when the plan allows dense
// passes (m > 4, 16-byte loads).
template <bool VEC, int ST>
static hipError_t launch_bp_v(const Plan& pl, const PassParams& pp, int j0, const float* S,
                              const uint8_t* act, float* gpart, int* touched, const Ctrl* ctrl,
                              hipStream_t st) {
    const int r = pl.m - j0;
    // every full group of 16 from j0 on in one launch
    if (r > 16 || (r == 16 && pl.m > 16))
        return launch_bp_t<16, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st, r / 16);
    const int mb = r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : r <= 8 ? 8 : 16;
    // m <= 16: the dense code rides in this launch; m > 16: k_backproj_dense
    const bool dense_here = j0 == 0 && pl.bp_thr <= kBpThrMax && pl.m <= 16;
    if constexpr (VEC) {
        if (dense_here && mb == 8) return launch_bp_t<8, VEC, ST, 1>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        if (dense_here && mb == 16) return launch_bp_t<16, VEC, ST, 1>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
    }
    if (dense_here) return hipErrorInvalidValue;   // the plan never allows this
    switch (mb) {
        case 1: return launch_bp_t<1, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        case 2: return launch_bp_t<2, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        case 4: return launch_bp_t<4, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        case 8: return launch_bp_t<8, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        default: return launch_bp_t<16, VEC, ST, 0>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
    }
}

// Component groups of at most 16 (the group's partial of g lives in registers).
hipError_t launch_backproj(const Plan& pl, const PassParams& pp, const float* S,
                           const uint8_t* act, float* gpart, int* touched, const Ctrl* ctrl,
                           hipStream_t st) {
    if (pl.bp_thr <= kBpThrMax && pl.m > 16) {
        hipError_t e;
        if (pl.dtype == GPSPCA_BF16)
            e = launch_bp_dense<kStBF16>(pl, pp, S, act, gpart, touched, ctrl, st);
        else if (pl.dtype == GPSPCA_F8E4M3)
            e = launch_bp_dense<kStF8>(pl, pp, S, act, gpart, touched, ctrl, st);
        else
            e = launch_bp_dense<kStF32>(pl, pp, S, act, gpart, touched, ctrl, st);
        if (e != hipSuccess) return e;
    }
    for (int j0 = 0; j0 < pl.m; j0 += (pl.m - j0 >= 16 && pl.m > 16) ? (pl.m - j0) / 16 * 16 : 16) {
        hipError_t e;
        if (pl.dtype == GPSPCA_BF16)
            e = launch_bp_v<true, kStBF16>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        else if (pl.dtype == GPSPCA_F8E4M3)
            e = launch_bp_v<true, kStF8>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        else if (pl.vec4)
            e = launch_bp_v<true, kStF32>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        else
            e = launch_bp_v<false, kStF32>(pl, pp, j0, S, act, gpart, touched, ctrl, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_colnorm(const PassParams& pp, int dtype, double* norms, int grid,
                          hipStream_t st) {
    if (dtype == GPSPCA_BF16) {
        hipLaunchKernelGGL((k_colnorm<true, kStBF16>), dim3(grid), dim3(256), 0, st, pp, norms);
    } else if (dtype == GPSPCA_F8E4M3) {
        hipLaunchKernelGGL((k_colnorm<true, kStF8>), dim3(grid), dim3(256), 0, st, pp, norms);
    } else {
        const bool vec = ((pp.lda & 3) == 0) && ((reinterpret_cast<uintptr_t>(pp.A) & 15) == 0);
        if (vec)
            hipLaunchKernelGGL((k_colnorm<true, kStF32>), dim3(grid), dim3(256), 0, st, pp, norms);
        else
            hipLaunchKernelGGL((k_colnorm<false, kStF32>), dim3(grid), dim3(256), 0, st, pp, norms);
    }
    return hipGetLastError();
}

}  // namespace gpspca
