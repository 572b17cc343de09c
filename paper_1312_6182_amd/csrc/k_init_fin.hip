// Default start and output kernels of the GP-SPCA power iteration.
//
// Default start: the m columns of largest norm, ordered by (-||a_i||, i), so
// ties go to the lower index; their polar factor (or normalization) is the
// starting point.  Selection is two-level: each workgroup keeps the top m of
// its column range, one workgroup merges the candidates.
//
// Outputs: Z = S with unit-norm columns (a column with empty support stays
// zero), the support as packed bit words, and X copied out of the internal
// padded buffer.
#include "gpspca_internal.h"
#include "storage.h"

namespace gpspca {

__device__ __forceinline__ bool better(double va, int64_t ia, double vb, int64_t ib) {
    if (ib < 0) return ia >= 0;
    if (ia < 0) return false;
    return va > vb || (va == vb && ia < ib);
}

// m rounds of a workgroup argmax over [b, e) of (val, idx) pairs.  The order
// "larger value, then lower index" is strict and total, so round r's winner
// is the best pair that comes after round r-1's winner in it: one comparison
// per pair and round, and any reduction order finds the same (unique) pair.
// Results in chosen_v / chosen_i (index -1 once the pairs run out).
__device__ __forceinline__ void wave_best(double& v, int64_t& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int64_t oi = __shfl_xor(i, o, 64);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

// Ranges of at most CAP pairs per thread are read once into registers (all
// loads issued together); longer ones are re-read every round.
template <int CAP>
__device__ void topm_block(int m, int64_t b, int64_t e, const double* __restrict__ val,
                           const int64_t* __restrict__ idx, double* chosen_v, int64_t* chosen_i,
                           double* rv, int64_t* ri) {
    const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6, nw = (nt + 63) >> 6;
    const bool in_regs = (e - b) <= (int64_t)CAP * nt;
    double pv[CAP];
    int64_t pi[CAP];
    if (in_regs) {
#pragma unroll
        for (int u = 0; u < CAP; ++u) {
            pv[u] = -INFINITY;
            pi[u] = -1;
        }
        if (e > b) {
#pragma unroll
            for (int u = 0; u < CAP; ++u) {
                const int64_t i = b + t + (int64_t)u * nt;
                const int64_t ic = i < e ? i : e - 1;   // in range; dropped below when i >= e
                const int64_t ci = idx ? idx[ic] : ic;
                const double cv = val[ic];
                pv[u] = (i < e && ci >= 0) ? cv : -INFINITY;
                pi[u] = (i < e) ? ci : -1;
            }
        }
    }
    double lv = INFINITY;   // the previous round's winner (none yet: every pair qualifies)
    int64_t li = -1;
    for (int r = 0; r < m; ++r) {
        double bv = -INFINITY;
        int64_t bi = -1;
        if (in_regs) {
#pragma unroll
            for (int u = 0; u < CAP; ++u) {
                if (pi[u] < 0) continue;
                const bool after = (r == 0) || better(lv, li, pv[u], pi[u]);
                if (after && better(pv[u], pi[u], bv, bi)) {
                    bv = pv[u];
                    bi = pi[u];
                }
            }
        } else {
            for (int64_t i = b + t; i < e; i += nt) {
                const int64_t ci = idx ? idx[i] : i;
                if (ci < 0) continue;
                const double cv = val[i];
                // after the previous winner in the order, and better than the best so far
                const bool after = (r == 0) || better(lv, li, cv, ci);
                if (after && better(cv, ci, bv, bi)) {
                    bv = cv;
                    bi = ci;
                }
            }
        }
        wave_best(bv, bi);
        if (lane == 0) {
            rv[wv] = bv;
            ri[wv] = bi;
        }
        __syncthreads();
        bv = rv[0];
        bi = ri[0];
        for (int w = 1; w < nw; ++w)
            if (better(rv[w], ri[w], bv, bi)) {
                bv = rv[w];
                bi = ri[w];
            }
        if (t == 0) {
            chosen_v[r] = bv;
            chosen_i[r] = bi;
        }
        lv = bv;
        li = bi;
        __syncthreads();
        if (bi < 0) {
            // pairs exhausted: the remaining rounds choose nothing
            for (int q = r + 1 + t; q < m; q += nt) {
                chosen_v[q] = -INFINITY;
                chosen_i[q] = -1;
            }
            __syncthreads();
            return;
        }
    }
}

__global__ __launch_bounds__(256) void k_topm_local(int64_t n, int m, const double* __restrict__ norms,
                                                    double* __restrict__ cv, int64_t* __restrict__ ci) {
    __shared__ double rv[256];
    __shared__ int64_t ri[256];
    __shared__ double chv[kMaxM];
    __shared__ int64_t chi[kMaxM];
    const int64_t b = n * blockIdx.x / gridDim.x, e = n * (blockIdx.x + 1) / gridDim.x;
    topm_block<8>(m, b, e, norms, nullptr, chv, chi, rv, ri);
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        cv[(size_t)blockIdx.x * m + r] = chv[r];
        ci[(size_t)blockIdx.x * m + r] = chi[r];
    }
}

// 1024 threads: the candidates (at most 256 workgroups x 64) fit 16 per thread.
__global__ __launch_bounds__(1024) void k_topm_final(int ncand, int m, const double* __restrict__ cv,
                                                     const int64_t* __restrict__ ci,
                                                     int64_t* __restrict__ idx) {
    __shared__ double rv[16];
    __shared__ int64_t ri[16];
    __shared__ double chv[kMaxM];
    __shared__ int64_t chi[kMaxM];
    topm_block<16>(m, 0, ncand, cv, ci, chv, chi, rv, ri);
    for (int r = threadIdx.x; r < m; r += blockDim.x) idx[r] = chi[r];
}

hipError_t launch_topm(const Plan& pl, const double* norms, double* cand_v, int64_t* cand_i,
                       int64_t* idx, hipStream_t st) {
    hipLaunchKernelGGL(k_topm_local, dim3(pl.topm_grid), dim3(256), 0, st, pl.n, pl.m, norms,
                       cand_v, cand_i);
    hipLaunchKernelGGL(k_topm_final, dim3(1), dim3(1024), 0, st, pl.topm_grid * pl.m, pl.m,
                       cand_v, cand_i, idx);
    return hipGetLastError();
}

// g64[j*p + r] = A[r, idx[j]] in FP64 (dequantized and scaled for 16/8-bit storage).
__global__ void k_gather(PassParams pp, int dtype, const int64_t* __restrict__ idx,
                         double* __restrict__ g64) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)pp.m * pp.p) return;
    const int j = (int)(e / pp.p), r = (int)(e % pp.p);
    const int64_t c = idx[j];
    double v;
    if (dtype == GPSPCA_BF16)
        v = (double)bf16_value(pp.Abf[c * pp.lda + r]) * (double)column_scale(pp, c);
    else if (dtype == GPSPCA_F8E4M3)
        v = (double)e4m3_value(pp.Af8[c * pp.lda + r]) * (double)column_scale(pp, c);
    else
        v = (double)pp.A[c * pp.lda + r];
    g64[e] = v;
}

hipError_t launch_gather(const Plan& pl, const PassParams& pp, const int64_t* idx, double* g64,
                         hipStream_t st) {
    const int64_t ne = (int64_t)pl.m * pl.p;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, pp,
                       pl.dtype, idx, g64);
    return hipGetLastError();
}

// Support words and per-block sums of s^2 per component.  S is row-major
// (n x m): thread t takes component t % m of word blockIdx.x * (256 / m) + t / m,
// so each load instruction of a wave reads consecutive components of a row.
__global__ __launch_bounds__(256) void k_fin_support(int64_t n, int m, const float* __restrict__ S,
                                                     uint32_t* __restrict__ support,
                                                     double* __restrict__ fin) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int wpb = 256 / m, j = t % m, k = t / m;
    const int64_t nw = (n + 31) / 32;
    const int64_t w = (int64_t)blockIdx.x * wpb + k;
    double ss = 0.0;
    if (k < wpb && w < nw) {
        uint32_t bits = 0;
        const int64_t i0 = w * 32;
        const int cnt = (int)((n - i0) < 32 ? (n - i0) : 32);
        for (int b = 0; b < cnt; ++b) {
            const float s = S[(i0 + b) * m + j];
            bits |= (s != 0.f ? 1u : 0u) << b;
            ss += (double)s * (double)s;
        }
        if (support) support[(size_t)j * nw + w] = bits;
    }
    red[t] = ss;
    __syncthreads();
    // per component, a fixed pairwise tree over the block's words
    for (int h = 1; h < wpb; h <<= 1) {
        if (k < wpb && (k & (2 * h - 1)) == 0 && k + h < wpb) red[t] += red[t + h * m];
        __syncthreads();
    }
    if (k == 0) fin[(size_t)blockIdx.x * m + j] = red[t];
}

// 1 / ||s_j|| from the per-block sums; grid (components), 256 threads: strided
// per-thread sums in block order, then a fixed tree.
__global__ __launch_bounds__(256) void k_fin_norm(int m, int nblk, const double* __restrict__ fin,
                                                  double* __restrict__ invn) {
    __shared__ double red[256];
    const int j = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblk; b += 256) s += fin[(size_t)b * m + j];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) invn[j] = red[0] > 0.0 ? 1.0 / sqrt(red[0]) : 0.0;
}

// Z[i + j*n] = S[i*m + j] * invn[j]  (invn == nullptr: plain transpose).  A
// workgroup transposes 64 rows of S through LDS: rows are read as one
// contiguous block, and each column j of Z is written as 64 consecutive
// values.
__global__ __launch_bounds__(256) void k_fin_z(int64_t n, int m, const float* __restrict__ S,
                                               const double* __restrict__ invn,
                                               float* __restrict__ Z) {
    __shared__ float tile[64 * (kMaxM + 1)];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int rows = (int)((n - i0) < 64 ? (n - i0) : 64);
    const int ld = m + 1;
    for (int e = t; e < rows * m; e += 256) tile[(e / m) * ld + e % m] = S[i0 * m + e];
    __syncthreads();
    for (int e = t; e < 64 * m; e += 256) {
        const int j = e >> 6, ii = e & 63;
        if (ii < rows) {
            const float s = tile[ii * ld + j];
            Z[(size_t)j * n + i0 + ii] = invn ? (float)((double)s * invn[j]) : s;
        }
    }
}

hipError_t launch_finalize(const Plan& pl, const float* S, double* fin, double* invn, float* Z,
                           uint32_t* support, hipStream_t st) {
    if (invn) {
        hipLaunchKernelGGL(k_fin_support, dim3(pl.fin_grid), dim3(256), 0, st, pl.n, pl.m, S,
                           support, fin);
        hipLaunchKernelGGL(k_fin_norm, dim3(pl.m), dim3(256), 0, st, pl.m, pl.fin_grid, fin, invn);
    }
    if (Z)
        hipLaunchKernelGGL(k_fin_z, dim3((unsigned)((pl.n + 63) / 64)), dim3(256), 0, st, pl.n,
                           pl.m, S, invn, Z);
    return hipGetLastError();
}

// Xout (p x m, leading dim p) <- Xint (leading dim ldx)
__global__ void k_copy_x(int m, int p, int ldx, const float* __restrict__ Xi, float* __restrict__ Xo) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)m * p) return;
    const int j = (int)(e / p), r = (int)(e % p);
    Xo[e] = Xi[(size_t)j * ldx + r];
}

// The same from the iterate of the last pass, X_{n_iter - 1}, which sits in
// Xa (n_iter odd) or Xb (n_iter even); nothing when no pass was made.
__global__ void k_copy_x_last(int m, int p, int ldx, const float* __restrict__ Xa,
                              const float* __restrict__ Xb, const Ctrl* __restrict__ ctrl,
                              float* __restrict__ Xo) {
    const int ni = ctrl->n_iter;
    if (ni < 1) return;
    const float* Xi = ((ni - 1) & 1) ? Xb : Xa;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)m * p) return;
    const int j = (int)(e / p), r = (int)(e % p);
    Xo[e] = Xi[(size_t)j * ldx + r];
}

hipError_t launch_copy_x_last(const Plan& pl, const float* Xa, const float* Xb, const Ctrl* ctrl,
                              float* Xout, hipStream_t st) {
    const int64_t ne = (int64_t)pl.m * pl.p;
    hipLaunchKernelGGL(k_copy_x_last, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, pl.m,
                       (int)pl.p, pl.ldx, Xa, Xb, ctrl, Xout);
    return hipGetLastError();
}

hipError_t launch_copy_x(const Plan& pl, const float* Xint, float* Xout, hipStream_t st) {
    const int64_t ne = (int64_t)pl.m * pl.p;
    hipLaunchKernelGGL(k_copy_x, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, pl.m,
                       (int)pl.p, pl.ldx, Xint, Xout);
    return hipGetLastError();
}

}  // namespace gpspca

namespace gpspca {

// Ascending list of the columns whose support bit is set for at least one
// component (the columns a frozen-support pass has to read).  One workgroup;
// each thread owns one 32-column word per round, and a workgroup prefix sum of
// the word populations places the thread's columns.
__global__ __launch_bounds__(1024) void k_mask_list(const uint32_t* __restrict__ mask,
                                                    int64_t words, int m, int64_t n,
                                                    int* __restrict__ list,
                                                    int* __restrict__ nlist) {
    __shared__ int wave_tot[16];
    __shared__ int base_s;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t == 0) base_s = 0;
    __syncthreads();
    for (int64_t w0 = 0; w0 < words; w0 += 1024) {
        const int64_t wi = w0 + t;
        uint32_t u = 0;
        if (wi < words) {
            for (int j = 0; j < m; ++j) u |= mask[(int64_t)j * words + wi];
            if (wi == words - 1 && (n & 31)) u &= (1u << (n & 31)) - 1u;
        }
        const int c = __popc(u);
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) wave_tot[wv] = incl;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 16; ++w) {
            const int v = wave_tot[w];
            if (w < wv) before += v;
            total += v;
        }
        int pos = base_s + before + incl - c;
        while (u) {
            const int b = __ffs(u) - 1;
            list[pos++] = (int)(wi * 32 + b);
            u &= u - 1u;
        }
        __syncthreads();
        if (t == 0) base_s += total;
        __syncthreads();
    }
    if (t == 0) *nlist = base_s;
}

hipError_t launch_mask_list(const uint32_t* mask, int64_t words, int m, int64_t n, int* list,
                            int* nlist, hipStream_t st) {
    hipLaunchKernelGGL(k_mask_list, dim3(1), dim3(1024), 0, st, mask, words, m, n, list, nlist);
    return hipGetLastError();
}

}  // namespace gpspca
