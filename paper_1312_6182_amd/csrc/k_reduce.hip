// Reduction, retraction and stopping kernels of the GP-SPCA power iteration.
//
// After a pass has produced per-workgroup partials of the ascent direction G
// (FP32) and per-wave objective partials (FP64), these kernels:
//   k_reduce_partials  sum the G partials in a fixed order (FP64 accumulation),
//   k_gram             finish G (FP64), and per row block the Gram matrices
//                      G^T G, G^T X_k, X_k^T X_k,
//   k_stop             (one workgroup) sum the objective F_k in fixed order, apply
//                      the stopping rule, and compute the retraction
//                      X_{k+1} = G Omega + X_k Psi:
//                        m = 1   Omega = 1/||g||           (unit sphere)
//                        block   Omega = (G^T G)^{-1/2}    (polar factor on the
//                                Stiefel manifold), from a cyclic Jacobi
//                                eigen-decomposition in FP64;
//                        dead components (empty support) are completed by the
//                        polar factor of the previous columns projected off the
//                        live part, expressed through the same Gram matrices,
//   k_apply            X_{k+1} = G Omega + X_k Psi, rounded to FP32.
// Every reduction runs in a fixed order, so results are bitwise reproducible.
#include "gpspca_internal.h"

namespace gpspca {

constexpr int LDM = kMaxM + 1;  // padded leading dimension of m x m LDS matrices

// Allow dynamic LDS beyond 64 KB (gfx950 has 160 KB per CU).
static void set_lds_limit(const void* fn) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();  // the attribute is advisory; do not leave a sticky error behind
}

// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t st) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<uint32_t*>(ptr), words);
    return hipGetLastError();
}

__device__ __forceinline__ void ctrl_reset_fields(Ctrl* ctrl, int max_iter, double tol) {
    ctrl->k = 0;
    ctrl->done = 0;
    ctrl->status = GPSPCA_OK;
    ctrl->n_iter = 0;
    ctrl->ndead = 0;
    ctrl->degenerate_seen = 0;
    ctrl->max_iter = max_iter;
    ctrl->warm = 0;
    ctrl->nact = 0;
    ctrl->tol = tol;
    ctrl->last_F = 0.0;
}

// Start of a solve in one launch: the control block reset (thread 0 of
// workgroup 0), the listed buffers cleared, and g64[j p + r] = X0[j ldx0 + r]
// in FP64 for j < m (m = 0: no X0).
__global__ __launch_bounds__(256) void k_start(Ctrl* ctrl, int max_iter, double tol, StartZero z,
                                               int m, int p, const float* __restrict__ X0,
                                               int ldx0, double* __restrict__ g64) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl_reset_fields(ctrl, max_iter, tol);
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t step = (size_t)gridDim.x * blockDim.x;
    for (int b = 0; b < z.n; ++b) {
        uint32_t* ptr = z.ptr[b];
        const size_t w = z.words[b];
        for (size_t i = i0; i < w; i += step) ptr[i] = 0u;
    }
    const size_t ne = (size_t)m * p;
    for (size_t e = i0; e < ne; e += step) {
        const size_t j = e / p, r = e % p;
        g64[e] = (double)X0[j * ldx0 + r];
    }
}

hipError_t launch_start(Ctrl* ctrl, int max_iter, double tol, const StartZero& z, int m, int p,
                        const float* X0, int ldx0, double* g64, hipStream_t st) {
    size_t most = X0 ? (size_t)m * p : 0;
    for (int i = 0; i < z.n; ++i) most = z.words[i] > most ? z.words[i] : most;
    size_t blocks = (most + 255) / 256;
    blocks = blocks < 1 ? 1 : blocks > 4096 ? 4096 : blocks;
    hipLaunchKernelGGL(k_start, dim3((unsigned)blocks), dim3(256), 0, st, ctrl, max_iter, tol, z,
                       X0 ? m : 0, p, X0, ldx0, g64);
    return hipGetLastError();
}

__global__ void k_ctrl_reset(Ctrl* ctrl, int max_iter, double tol) {
    if (threadIdx.x == 0) {
        ctrl->k = 0;
        ctrl->done = 0;
        ctrl->status = GPSPCA_OK;
        ctrl->n_iter = 0;
        ctrl->ndead = 0;
        ctrl->degenerate_seen = 0;
        ctrl->max_iter = max_iter;
        ctrl->warm = 0;
        ctrl->nact = 0;
        ctrl->tol = tol;
        ctrl->last_F = 0.0;
    }
}

hipError_t launch_ctrl_reset(Ctrl* ctrl, int max_iter, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, ctrl, max_iter, tol);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// l1[y][e] = sum_{c in chunk y} gpart[c][e]  (e < m*ldx), skipping untouched
// partials; chunks are contiguous ranges of the partial index.
__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ gpart,
                                                         const int* __restrict__ touched,
                                                         int npart, int nsplit, int64_t ne,
                                                         double* __restrict__ l1,
                                                         const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    const int y = blockIdx.y;
    const int c0 = (int)((int64_t)npart * y / nsplit), c1 = (int)((int64_t)npart * (y + 1) / nsplit);
    // this split's touched partials as an ascending list in LDS, built once
    // (a partial that no workgroup wrote is neither read nor added)
    __shared__ int plist[1024];
    __shared__ int wcnt[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const bool staged = touched && (c1 - c0) <= 1024;
    int nlist = 0;
    if (staged) {
        for (int b = 0; b < c1 - c0; b += 256) {
            const int i = b + t;
            const bool on = i < c1 - c0 && touched[c0 + i] != 0;
            const uint64_t bal = __ballot(on);
            if (lane == 0) wcnt[wv] = __popcll(bal);
            __syncthreads();
            int before = nlist;
            for (int w = 0; w < wv; ++w) before += wcnt[w];
            if (on) plist[before + __popcll(bal & ((1ull << lane) - 1ull))] = c0 + i;
            nlist += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
            __syncthreads();
        }
    }
    const int64_t e = (int64_t)blockIdx.x * 256 + t;
    if (e >= ne) return;
    double s = 0.0;
    int c = c0;
    if (staged) {
        // in list order (ascending c); the loads of 8 partials are issued
        // together (past the end the last one is re-read and not added)
        for (int q = 0; q < nlist; q += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = gpart[(size_t)plist[q + u < nlist ? q + u : nlist - 1] * ne + e];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u < nlist) s += (double)v[u];
        }
        c = c1;
    } else if (!touched) {
        for (; c + 4 <= c1; c += 4) {
            const float v0 = gpart[(size_t)c * ne + e];
            const float v1 = gpart[(size_t)(c + 1) * ne + e];
            const float v2 = gpart[(size_t)(c + 2) * ne + e];
            const float v3 = gpart[(size_t)(c + 3) * ne + e];
            s += (double)v0;
            s += (double)v1;
            s += (double)v2;
            s += (double)v3;
        }
    }
    for (; c < c1; ++c)
        if (!touched || touched[c]) s += (double)gpart[(size_t)c * ne + e];
    l1[(size_t)y * ne + e] = s;
}

hipError_t launch_reduce_partials(const Plan& pl, const float* gpart, const int* touched,
                                  double* l1, const Ctrl* ctrl, hipStream_t st) {
    const int64_t ne = (int64_t)pl.m * pl.ldx;
    dim3 grid((unsigned)((ne + 255) / 256), (unsigned)pl.red_split);
    hipLaunchKernelGGL(k_reduce_partials, grid, dim3(256), 0, st, gpart, touched, pl.npart,
                       pl.red_split, ne, l1, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row block r0..r0+nr: g_r = sum_y l1[y][.][r] (fixed order) -> g64 (p x m,
// leading dim p); partial Gram matrices over the block ->
// gram[blk][0|1|2][m*m] = G^T G, G^T X, X^T X.
// G^T G, G^T X and X^T X of one row block held in LDS (gt, xt: rows x (m+1)),
// R x R entries per thread; rows are added in order, as in the untiled loop.
template <int R>
__device__ __forceinline__ void gram_tiles(const double* gt, const double* xt, int mp, int nr,
                                           int m, int with_x, int t, double* out) {
    const int ta = t >> 4, tb = t & 15, mm = m * m;
    int ia[R], ib[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        ia[i] = (ta + 16 * i < m) ? ta + 16 * i : m - 1;
        ib[i] = (tb + 16 * i < m) ? tb + 16 * i : m - 1;
    }
    double sgg[R][R], sgx[R][R], sxx[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) sgg[i][k] = sgx[i][k] = sxx[i][k] = 0.0;
    for (int rr = 0; rr < nr; ++rr) {
        const double* gr = gt + rr * mp;
        const double* xr = xt + rr * mp;
        double ga[R], gb[R], xa[R], xb[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            ga[i] = gr[ia[i]];
            gb[i] = gr[ib[i]];
            xa[i] = xr[ia[i]];
            xb[i] = xr[ib[i]];
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int k = 0; k < R; ++k) {
                sgg[i][k] += ga[i] * gb[k];
                sgx[i][k] += ga[i] * xb[k];
                sxx[i][k] += xa[i] * xb[k];
            }
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int a = ta + 16 * i, b = tb + 16 * k;
            if (a < m && b < m) {
                const int e = a * m + b;
                out[e] = sgg[i][k];
                out[mm + e] = with_x == 1 ? sgx[i][k] : 0.0;
                out[2 * mm + e] = with_x == 1 ? sxx[i][k] : 0.0;
            }
        }
}

__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ l1, int nsplit, int m,
                                              int ldx, int p, int rows, const float* __restrict__ X,
                                              int with_x, double* __restrict__ g64,
                                              double* __restrict__ gram,
                                              const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    extern __shared__ double sh[];
    const int mp = m + 1;
    double* gt = sh;                         // rows x (m+1)
    double* xt = sh + (size_t)rows * mp;     // rows x (m+1)
    const int r0 = blockIdx.x * rows;
    const int nr = (p - r0 < rows) ? p - r0 : rows;
    const int t = threadIdx.x;
    const size_t ne = (size_t)m * ldx;
    for (int e = t; e < nr * m; e += blockDim.x) {
        const int rr = e % nr, j = e / nr;
        double s;
        if (l1) {
            // in order of y; the loads of 8 splits are issued together
            const double* src = l1 + (size_t)j * ldx + r0 + rr;
            s = 0.0;
            int y = 0;
            for (; y + 8 <= nsplit; y += 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(y + u) * ne];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
            for (; y < nsplit; ++y) s += src[(size_t)y * ne];
            g64[(size_t)j * p + r0 + rr] = s;
        } else {
            s = g64[(size_t)j * p + r0 + rr];
        }
        gt[rr * mp + j] = s;
        xt[rr * mp + j] = (with_x == 1) ? (double)X[(size_t)j * ldx + r0 + rr] : 0.0;
    }
    __syncthreads();
    const int mm = m * m;
    double* out = gram + (size_t)blockIdx.x * 3 * mm;
    // Few entries (small m, or the diagonal only on a gamma path): every entry
    // is summed by S row slices in parallel, then a fixed-order tree adds the
    // slices, instead of one thread walking all rows.
    const int nent = (with_x == 2) ? m : 3 * mm;
    if (nent <= 128) {
        __shared__ double red[256];
        int S = 1;
        while (2 * S * nent <= (int)blockDim.x && S < 64) S *= 2;
        if (t < nent * S) {
            const int e = t % nent, sl = t / nent;
            double acc = 0.0;
            if (with_x == 2) {
                for (int rr = sl; rr < nr; rr += S) acc += gt[rr * mp + e] * gt[rr * mp + e];
            } else {
                const int which = e / mm, ab = e % mm, a = ab / m, b = ab % m;
                const double* u = which == 2 ? xt : gt;
                const double* w = which == 0 ? gt : xt;
                if (which == 0 || with_x == 1)
                    for (int rr = sl; rr < nr; rr += S) acc += u[rr * mp + a] * w[rr * mp + b];
            }
            red[sl * nent + e] = acc;
        }
        __syncthreads();
        for (int h = S / 2; h >= 1; h /= 2) {
            if (t < nent * h) red[t] += red[t + h * nent];
            __syncthreads();
        }
        if (t < nent) {
            if (with_x == 2) out[t * m + t] = red[t];
            else out[t] = red[t];
        }
        return;
    }
    if (with_x == 2) {  // independent columns (gamma path): only ||g_j||^2 is needed
        for (int a = t; a < m; a += blockDim.x) {
            double sgg = 0.0;
            for (int rr = 0; rr < nr; ++rr) sgg += gt[rr * mp + a] * gt[rr * mp + a];
            out[a * m + a] = sgg;
        }
        return;
    }
    if (m > 16 && blockDim.x == 256) {
        // register tiles: thread (ta, tb) of a 16 x 16 grid owns entries
        // (ta + 16 i, tb + 16 k), i, k < R, of the three products, so a row
        // costs 4R LDS reads for 3 R^2 multiply-adds
        if (m <= 32) gram_tiles<2>(gt, xt, mp, nr, m, with_x, t, out);
        else gram_tiles<4>(gt, xt, mp, nr, m, with_x, t, out);
        return;
    }
    for (int e = t; e < mm; e += blockDim.x) {
        const int a = e / m, b = e % m;
        double sgg = 0.0, sgx = 0.0, sxx = 0.0;
        for (int rr = 0; rr < nr; ++rr) {
            const double ga = gt[rr * mp + a];
            sgg += ga * gt[rr * mp + b];
            if (with_x == 1) {
                sgx += ga * xt[rr * mp + b];
                sxx += xt[rr * mp + a] * xt[rr * mp + b];
            }
        }
        out[e] = sgg;
        out[mm + e] = sgx;
        out[2 * mm + e] = sxx;
    }
}

hipError_t launch_gram(const Plan& pl, const double* l1, int nsplit, const float* X, int with_x,
                       double* g64, double* gram, const Ctrl* ctrl, hipStream_t st) {
    const size_t shm = (size_t)2 * pl.gram_rows * (pl.m + 1) * sizeof(double);
    static const bool lds_once = (set_lds_limit((const void*)k_gram), true);
    (void)lds_once;
    hipLaunchKernelGGL(k_gram, dim3(pl.gram_grid), dim3(256), shm, st, l1, nsplit, pl.m, pl.ldx,
                       (int)pl.p, pl.gram_rows, X, with_x, g64, gram, ctrl);
    return hipGetLastError();
}

// Final fixed-order reduction of the per-row-block Gram partials into the
// coefficient scratch: coef[2mm + e] = sum_g gram[g][e] for e < nent.
// Each workgroup owns EPB = 256 / S entries; S slices per entry sum the
// partials g = sl, sl + S, ... and a fixed-order tree adds the slices.
// Blocks past the Gram entries (fsum != NULL) each sum one component's
// objective and support-size partials: fsum[j] = sum_w fpart[j nwp + w],
// fsum[m + j] = sum_w nnzpart[j nwp + w] (thread slices in order, then a fixed
// tree), so the one-workgroup stop kernel reads 2m numbers.
__global__ __launch_bounds__(256) void k_gram_sum(int nent, int mm, int ngram, int S,
                                                  const double* __restrict__ gram,
                                                  double* __restrict__ coef,
                                                  const double* __restrict__ fpart,
                                                  const int* __restrict__ nnzpart, int nwp,
                                                  int m, double* __restrict__ fsum,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double red[256];
    __shared__ long long redc[256];
    const int t = threadIdx.x, epb = 256 / S;
    const int nblk = (nent + epb - 1) / epb;
    if ((int)blockIdx.x >= nblk) {
        const int j = blockIdx.x - nblk;
        double sf = 0.0;
        long long sc = 0;
        for (int w0 = t; w0 < nwp; w0 += 8 * 256) {
            double v[8];
            int c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int w = w0 + u * 256;
                const int wc = w < nwp ? w : nwp - 1;
                v[u] = fpart[(size_t)j * nwp + wc];
                c[u] = nnzpart[(size_t)j * nwp + wc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (w0 + u * 256 < nwp) {
                    sf += v[u];
                    sc += c[u];
                }
        }
        red[t] = sf;
        redc[t] = sc;
        __syncthreads();
        for (int hh = 128; hh >= 1; hh >>= 1) {
            if (t < hh) {
                red[t] += red[t + hh];
                redc[t] += redc[t + hh];
            }
            __syncthreads();
        }
        if (t == 0) {
            fsum[j] = red[0];
            fsum[m + j] = (double)redc[0];
        }
        return;
    }
    const int el = t % epb, sl = t / epb;
    const int e = blockIdx.x * epb + el;
    double s = 0.0;
    if (e < nent) {
        // in order of g; the loads of 8 terms are issued together (indices past
        // the end re-read the last term and are not added)
        const double* gp = gram + e;
        for (int g0 = sl; g0 < ngram; g0 += 8 * S) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int g = g0 + u * S;
                v[u] = gp[(size_t)(g < ngram ? g : ngram - 1) * 3 * mm];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (g0 + u * S < ngram) s += v[u];
        }
    }
    red[t] = s;
    __syncthreads();
    for (int h = S / 2; h >= 1; h /= 2) {
        if (sl < h) red[t] += red[t + h * epb];
        __syncthreads();
    }
    if (sl == 0 && e < nent) coef[2 * mm + e] = red[t];
}

hipError_t launch_gram_sum(const Plan& pl, int nent, int ngram, const double* gram, double* coef,
                           const Ctrl* ctrl, hipStream_t st, const double* fpart,
                           const int* nnzpart, double* fsum) {
    const int mm = pl.m * pl.m;
    // slices per entry: enough to shorten the serial chains, while keeping at
    // least a few workgroups busy
    int S = 1;
    while (S < 64 && S * 8 <= ngram && (nent * 2 * S + 255) / 256 <= 64) S *= 2;
    const int epb = 256 / S;
    const int blocks = (nent + epb - 1) / epb + (fsum ? pl.m : 0);
    hipLaunchKernelGGL(k_gram_sum, dim3(blocks), dim3(256), 0, st, nent, mm, ngram, S, gram, coef,
                       fpart, nnzpart, pl.nwave_part, pl.m, fsum, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused partial reduction + Gram for m <= 16: one workgroup per 64 rows.
// Thread (row rr, slice sl) sums the partials c = sl, sl+4, ... of its row for
// every component, the four slices are added in order 0..3 (fixed order), the
// row of G is written in FP64, and the block's contributions to G^T G, G^T X,
// X^T X (or only the diagonal of G^T G, with_x == 2) go to gram[block].
template <int MB>
__global__ __launch_bounds__(256) void k_reduce_gram(const float* __restrict__ gpart,
                                                     const int* __restrict__ touched, int npart,
                                                     int m, int ldx, int p,
                                                     const float* __restrict__ X, int with_x,
                                                     double* __restrict__ g64,
                                                     double* __restrict__ gram,
                                                     const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int MP = MB + 1;
    __shared__ double part[4][64][MP];
    __shared__ double gt[64][MP];
    __shared__ double xt[64][MP];
    __shared__ int plist[1024];
    __shared__ int wcnt[4];
    const int t = threadIdx.x, rr = t & 63, sl = t >> 6;
    const int r0 = blockIdx.x * 64;
    const int r = r0 + rr;
    const int nr = (p - r0 < 64) ? p - r0 : 64;
    const size_t stride = (size_t)m * ldx;
    // ascending list of the partials that hold data (all of them without flags),
    // built in parallel so that the sums below never wait on a flag
    int nlist = 0;
    for (int c0 = 0; c0 < npart; c0 += 256) {
        const int c = c0 + t;
        const bool on = c < npart && (!touched || touched[c] != 0);
        const uint64_t bal = __ballot(on);
        if ((t & 63) == 0) wcnt[sl] = __popcll(bal);
        __syncthreads();
        int before = nlist;
        for (int w = 0; w < sl; ++w) before += wcnt[w];
        if (on && before + __popcll(bal & ((1ull << (t & 63)) - 1ull)) < 1024)
            plist[before + __popcll(bal & ((1ull << (t & 63)) - 1ull))] = c;
        nlist += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
    double g[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) g[j] = 0.0;
    // component offsets: components >= m re-read component m - 1 (a valid
    // address) and are dropped by a select, so the loads stay unconditional and
    // are issued together instead of one branch and one wait per component
    size_t joff[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) joff[j] = (size_t)(j < m ? j : m - 1) * ldx + r;
    if (r < p && nlist <= 1024) {
        int e = sl;
        for (; e + 12 < nlist; e += 16) {
            float v[4][MB];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float* src = gpart + (size_t)plist[e + 4 * u] * stride;
#pragma unroll
                for (int j = 0; j < MB; ++j) v[u][j] = src[joff[j]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int j = 0; j < MB; ++j) g[j] += (j < m) ? (double)v[u][j] : 0.0;
        }
        for (; e < nlist; e += 4) {
            float v[MB];
            const float* src = gpart + (size_t)plist[e] * stride;
#pragma unroll
            for (int j = 0; j < MB; ++j) v[j] = src[joff[j]];
#pragma unroll
            for (int j = 0; j < MB; ++j) g[j] += (j < m) ? (double)v[j] : 0.0;
        }
    } else if (r < p) {
        // more than 1024 partials: walk the flags directly
        for (int c = sl; c < npart; c += 4) {
            if (touched && !touched[c]) continue;
            float v[MB];
            const float* src = gpart + (size_t)c * stride;
#pragma unroll
            for (int j = 0; j < MB; ++j) v[j] = src[joff[j]];
#pragma unroll
            for (int j = 0; j < MB; ++j) g[j] += (j < m) ? (double)v[j] : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < MB; ++j) part[sl][rr][j] = g[j];
    __syncthreads();
    if (sl == 0) {
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const double v = ((part[0][rr][j] + part[1][rr][j]) + part[2][rr][j]) + part[3][rr][j];
            gt[rr][j] = v;
            if (r < p && j < m) g64[(size_t)j * p + r] = v;
            xt[rr][j] = (with_x == 1 && r < p && j < m) ? (double)X[(size_t)j * ldx + r] : 0.0;
        }
    }
    __syncthreads();
    const int mm = m * m;
    double* out = gram + (size_t)blockIdx.x * 3 * mm;
    if (with_x == 2) {
        for (int a = t; a < m; a += 256) {
            double sgg = 0.0;
            for (int k = 0; k < nr; ++k) sgg += gt[k][a] * gt[k][a];
            out[a * m + a] = sgg;
        }
        return;
    }
    for (int e = t; e < 3 * mm; e += 256) {
        const int which = e / mm, ab = e % mm, a = ab / m, b = ab % m;
        double s2 = 0.0;
        if (which == 0)
            for (int k = 0; k < nr; ++k) s2 += gt[k][a] * gt[k][b];
        else if (which == 1)
            for (int k = 0; k < nr; ++k) s2 += gt[k][a] * xt[k][b];
        else
            for (int k = 0; k < nr; ++k) s2 += xt[k][a] * xt[k][b];
        out[e] = s2;
    }
}

hipError_t launch_reduce_gram(const Plan& pl, const float* gpart, const int* touched,
                              const float* X, int with_x, double* g64, double* gram,
                              const Ctrl* ctrl, hipStream_t st) {
    const int grid = (int)((pl.p + 63) / 64);
#define GPSPCA_RG(MB)                                                                        \
    hipLaunchKernelGGL(k_reduce_gram<MB>, dim3(grid), dim3(256), 0, st, gpart, touched,     \
                       pl.npart, pl.m, pl.ldx, (int)pl.p, X, with_x, g64, gram, ctrl)
    if (pl.m <= 1) GPSPCA_RG(1);
    else if (pl.m <= 2) GPSPCA_RG(2);
    else if (pl.m <= 4) GPSPCA_RG(4);
    else if (pl.m <= 8) GPSPCA_RG(8);
    else GPSPCA_RG(16);
#undef GPSPCA_RG
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric eigen-decomposition by the cyclic Jacobi method with a parallel
// (round-robin) ordering: each step applies msz/2 disjoint plane rotations.
// a (msz x msz, leading dim LDM, LDS) is diagonalized in place; v receives the
// eigenvectors (columns).  With `warm`, v already holds an orthogonal V0 and a
// holds V0^T M V0: the rotations continue from there (V <- V0 J ...).
//
// Layout: during a sweep the matrix is kept in slot coordinates.  With mm =
// msz rounded up to even (an odd size gets a zero padding row and column that
// never rotates), step r of the round-robin schedule pairs slot k with slot
// mm - 1 - k, and slot s holds index 0 (s = 0) or 1 + (s - 1 + r) mod (mm - 1).
// Moving to step r + 1 then shifts the contents of every slot s >= 2 to s - 1
// and slot 1 to mm - 1, the same permutation at every step, so each step reads
// its pairs at fixed addresses and writes the rotated entries straight to
// their places for the next step: every thread's LDS offsets are computed once
// for the whole eigensolve.  A sweep is mm - 1 steps, after which the slots
// are back in index order.  Only one entry of each symmetric pair is kept
// during the sweeps (the one whose row slot belongs to the pair of lower
// number, or the upper one within a pair); the other is filled in at the end.
//
// A step: threads k < mm/2 compute the rotation of pair k while every thread
// loads its items (2 x 2 blocks of A over a pair of pairs, upper half only,
// and rows of V over one pair); then each item applies its rotations
// (A <- R A R^T, V <- V R^T) and stores the results at the next step's slots.
//
// A pair is rotated while |a_pq| > 2^-16 sqrt(|a_pp a_qq|) (the relative test,
// which keeps the small eigenvalues of a graded matrix accurate); the inverse
// square root is then built with the first-order correction of the remaining
// off-diagonal (inv_sqrt_from_eig), which leaves an error of second order,
// far below the FP32 of the retracted X.  The rotated pair's off-diagonal entry is
// set to zero exactly, as the rotation makes it: computed, it would keep a
// rounding residue of about 2^-52 max(a_pp, a_qq), which the relative test
// would chase without end when a_pp / a_qq is large.
// a and v need mm rows.  Executed by the whole workgroup.

// Items per thread of a Jacobi step; the kernels that call jacobi_eig launch
// at least jacobi_threads(m) threads.
constexpr int kItems = 3;

// Threads for an m x m Jacobi step: m > 32: 1024 (at most 32 x 33 / 2 blocks
// of A + 64 x 32 rows of V = 2576 items); m > 16: 512 (at most 648); m > 8: 256
// (at most 164); else one wave (at most 42 items and 16 entries of a product,
// and a barrier of a single wave costs almost nothing).
static int jacobi_threads(int m) { return m > 32 ? 1024 : m > 16 ? 512 : m > 8 ? 256 : 64; }

__device__ __forceinline__ int jac_pidx(int s, int mm) { return s < mm / 2 ? s : mm - 1 - s; }

// slot that receives slot s's contents at the next step
__device__ __forceinline__ int jac_next(int s, int mm) {
    return s == 0 ? 0 : (s == 1 ? mm - 1 : s - 1);
}

// offset of the kept entry of the symmetric pair (u, w)
__device__ __forceinline__ int jac_kept(int u, int w, int mm) {
    const int pu = jac_pidx(u, mm), pw = jac_pidx(w, mm);
    const bool swap = pu > pw || (pu == pw && u > w);
    return swap ? w * LDM + u : u * LDM + w;
}

__device__ void jacobi_eig(double* a, double* v, int msz, double* rot, bool warm = false) {
    const int t = threadIdx.x, nt = blockDim.x;
    // |a_pq| > 2^-16 sqrt(|a_pp a_qq|), tested squared (no square root)
    constexpr double kTol2 = 2.3283064365386963e-10;  // 2^-32
    if (!warm) {
        for (int e = t; e < msz * msz; e += nt) {
            const int i = e / msz, j = e % msz;
            v[i * LDM + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    if (msz < 2) {
        __syncthreads();
        return;
    }
    const int mm = msz + (msz & 1), half = mm / 2;
    if (msz & 1) {
        for (int e = t; e < mm; e += nt) {
            a[msz * LDM + e] = 0.0;
            a[e * LDM + msz] = 0.0;
        }
        for (int e = t; e < msz; e += nt) v[e * LDM + msz] = 0.0;
    }
    // items: upper blocks (k1 <= k2) of A, then rows of V; thread t owns
    // items t, t + nt, ... (at most kItems: blockDim.x is chosen for that)
    const int nA = half * (half + 1) / 2, nitem = nA + msz * half;
    int kind[kItems];     // 0 none, 1 block of A, 2 diagonal block of A, 3 row of V
    int rk1[kItems], rk2[kItems];
    int ld[kItems][4], sto[kItems][4];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int e = t + u * nt;
        kind[u] = 0;
        rk1[u] = rk2[u] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) ld[u][q] = sto[u][q] = 0;
        if (e >= nitem) continue;
        if (e < nA) {
            int k1 = 0, rem = e;
            while (rem >= half - k1) {
                rem -= half - k1;
                ++k1;
            }
            const int k2 = k1 + rem;
            const int P1 = k1, Q1 = mm - 1 - k1, P2 = k2, Q2 = mm - 1 - k2;
            const int nP1 = jac_next(P1, mm), nQ1 = jac_next(Q1, mm);
            const int nP2 = jac_next(P2, mm), nQ2 = jac_next(Q2, mm);
            rk1[u] = k1;
            rk2[u] = k2;
            if (k1 < k2) {
                kind[u] = 1;
                ld[u][0] = P1 * LDM + P2;
                ld[u][1] = P1 * LDM + Q2;
                ld[u][2] = Q1 * LDM + P2;
                ld[u][3] = Q1 * LDM + Q2;
                sto[u][0] = jac_kept(nP1, nP2, mm);
                sto[u][1] = jac_kept(nP1, nQ2, mm);
                sto[u][2] = jac_kept(nQ1, nP2, mm);
                sto[u][3] = jac_kept(nQ1, nQ2, mm);
            } else {
                kind[u] = 2;
                ld[u][0] = P1 * LDM + P1;
                ld[u][1] = P1 * LDM + Q1;
                ld[u][3] = Q1 * LDM + Q1;
                sto[u][0] = jac_kept(nP1, nP1, mm);
                sto[u][1] = jac_kept(nP1, nQ1, mm);
                sto[u][3] = jac_kept(nQ1, nQ1, mm);
            }
        } else {
            const int f = e - nA, row = f % msz, k = f / msz;
            const int P = k, Q = mm - 1 - k;
            kind[u] = 3;
            rk1[u] = k;
            ld[u][0] = row * LDM + P;
            ld[u][1] = row * LDM + Q;
            sto[u][0] = row * LDM + jac_next(P, mm);
            sto[u][1] = row * LDM + jac_next(Q, mm);
        }
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        // a sweep that would apply no rotation ends the iteration.  Every pair
        // is tested at once before the sweep (the slots are in index order
        // here): if none qualifies, no step of the sweep would rotate.
        int need = 0;
        for (int e = t; e < msz * msz; e += nt) {
            const int i = e / msz, j = e % msz;
            if (i != j && jac_kept(i, j, mm) == i * LDM + j) {
                const double apq = a[i * LDM + j];
                need |= (apq * apq > kTol2 * fabs(a[i * LDM + i] * a[j * LDM + j]) &&
                         fabs(apq) > 1e-300) ? 1 : 0;
            }
        }
        if (!__syncthreads_or(need)) break;
        for (int r = 0; r < mm - 1; ++r) {
            // phase 1: the rotations of this step, and every item's loads
            if (t < half) {
                const int P = t, Q = mm - 1 - t;
                const double apq = a[P * LDM + Q];
                const double app = a[P * LDM + P], aqq = a[Q * LDM + Q];
                double c = 1.0, sn = 0.0;
                if (apq * apq > kTol2 * fabs(app * aqq) && fabs(apq) > 1e-300) {
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = rsqrt(1.0 + tt * tt);
                    sn = tt * c;
                }
                rot[2 * t] = c;
                rot[2 * t + 1] = sn;
            }
            double x[kItems][4];
#pragma unroll
            for (int u = 0; u < kItems; ++u) {
                x[u][0] = x[u][1] = x[u][2] = x[u][3] = 0.0;
                if (kind[u] == 1) {
                    x[u][0] = a[ld[u][0]];
                    x[u][1] = a[ld[u][1]];
                    x[u][2] = a[ld[u][2]];
                    x[u][3] = a[ld[u][3]];
                } else if (kind[u] == 2) {
                    x[u][0] = a[ld[u][0]];
                    x[u][1] = a[ld[u][1]];
                    x[u][3] = a[ld[u][3]];
                } else if (kind[u] == 3) {
                    x[u][0] = v[ld[u][0]];
                    x[u][1] = v[ld[u][1]];
                }
            }
            __syncthreads();
            // phase 2: rotate and store at the next step's slots
#pragma unroll
            for (int u = 0; u < kItems; ++u) {
                if (kind[u] == 0) continue;
                const double c1 = rot[2 * rk1[u]], s1 = rot[2 * rk1[u] + 1];
                if (kind[u] == 3) {
                    const double vp = x[u][0], vq = x[u][1];
                    v[sto[u][0]] = c1 * vp - s1 * vq;
                    v[sto[u][1]] = s1 * vp + c1 * vq;
                    continue;
                }
                const double c2 = rot[2 * rk2[u]], s2 = rot[2 * rk2[u] + 1];
                const double x00 = x[u][0], x01 = x[u][1], x11 = x[u][3];
                const double x10 = (kind[u] == 2) ? x01 : x[u][2];
                // rows
                const double r00 = c1 * x00 - s1 * x10, r01 = c1 * x01 - s1 * x11;
                const double r10 = s1 * x00 + c1 * x10, r11 = s1 * x01 + c1 * x11;
                // columns
                a[sto[u][0]] = c2 * r00 - s2 * r01;
                if (kind[u] == 1) {
                    a[sto[u][1]] = s2 * r00 + c2 * r01;
                    a[sto[u][2]] = c2 * r10 - s2 * r11;
                } else {
                    // the rotated pair's off-diagonal is zero by construction
                    a[sto[u][1]] = (s1 != 0.0) ? 0.0 : x01;
                }
                a[sto[u][3]] = s2 * r10 + c2 * r11;
            }
            __syncthreads();
        }
    }
    // fill in the other entry of every symmetric pair
    for (int e = t; e < msz * msz; e += nt) {
        const int i = e / msz, j = e % msz;
        const int kp = jac_kept(i, j, mm);
        if (kp != i * LDM + j) a[i * LDM + j] = a[kp];
    }
    __syncthreads();
}

// C = op(A) op(B) for n x n matrices in LDS (leading dim LDM), op(X) = X or
// X^T.  With h = ceil(n/2), thread t = ii h + jj computes the four entries
// (ii | ii + h) x (jj | jj + h) of C in registers, summing over k in order
// (h^2 <= blockDim.x: jacobi_threads): the lanes of a wave then read
// consecutive entries of B (and share those of A), free of LDS bank
// conflicts.  C is written after a barrier, so it may be A or B.  Executed by
// the whole workgroup.
template <bool TA, bool TB>
__device__ void lds_gemm(int n, const double* A, const double* B, double* C) {
    const int t = threadIdx.x, h = (n + 1) / 2;
    const bool mine = t < h * h;
    const int ii = mine ? t / h : 0, jj = mine ? t % h : 0;
    const int i1 = ii + h < n ? ii + h : ii, j1 = jj + h < n ? jj + h : jj;
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
    if (mine) {
        for (int k = 0; k < n; ++k) {
            const double a0 = TA ? A[k * LDM + ii] : A[ii * LDM + k];
            const double a1 = TA ? A[k * LDM + i1] : A[i1 * LDM + k];
            const double b0 = TB ? B[jj * LDM + k] : B[k * LDM + jj];
            const double b1 = TB ? B[j1 * LDM + k] : B[k * LDM + j1];
            c00 += a0 * b0;
            c01 += a0 * b1;
            c10 += a1 * b0;
            c11 += a1 * b1;
        }
    }
    __syncthreads();
    if (mine) {
        C[ii * LDM + jj] = c00;
        if (jj + h < n) C[ii * LDM + jj + h] = c01;
        if (ii + h < n) C[(ii + h) * LDM + jj] = c10;
        if (ii + h < n && jj + h < n) C[(ii + h) * LDM + jj + h] = c11;
    }
    __syncthreads();
}

// out = V Y V^T ~ (V a V^T)^{-1/2} from the Jacobi result: a = V^T M V is
// diagonal up to off-diagonal entries below the stopping tolerance.  Y is the
// inverse square root of a to first order in its off-diagonal (the
// Daleckii-Krein formula): Y_ii = a_ii^{-1/2}, and for i != j
//   Y_ij = f[a_ii, a_jj] a_ij,  f[x, y] = (x^{-1/2} - y^{-1/2}) / (x - y)
//        = -1 / (sqrt(x) sqrt(y) (sqrt(x) + sqrt(y))),
// a divided difference that stays finite for equal diagonal entries.  The
// error left is second order in the relative off-diagonal e (measured below
// 250 e^2 on the retracted X: 6e-8 at e = 2^-16, the FP32 rounding of X), so
// the sweeps stop there.
// Eigenvalues below (msz * eps)^2 * lam_max count as zero (their row and
// column of Y are dropped) and set *rankdef.  a is overwritten.
__device__ void inv_sqrt_from_eig(double* a, const double* v, double* out, int msz,
                                  double* lam, int* rankdef) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int ne = msz * msz;
    // every thread finds the largest eigenvalue; thread i inverts the root of
    // eigenvalue i
    double lmax = 0.0;
    for (int i = 0; i < msz; ++i) lmax = fmax(lmax, a[i * LDM + i]);
    const double thr = lmax * ((double)msz * 2.220446049250313e-16) * ((double)msz * 2.220446049250313e-16);
    int rd = !(lmax > 0.0);
    for (int i = t; i < msz; i += nt) {
        const double l = a[i * LDM + i];
        if (l > thr && l > 0.0) lam[i] = 1.0 / sqrt(l);
        else { lam[i] = 0.0; rd = 1; }
    }
    rd = __syncthreads_or(rd);
    if (t == 0) *rankdef = rd;
    // Y in place of a: with l_i = a_ii^{-1/2}, f[a_ii, a_jj] = -(l_i l_j)^2 / (l_i + l_j)
    for (int e = t; e < ne; e += nt) {
        const int i = e / msz, j = e % msz;
        const double li = lam[i], lj = lam[j];
        double y;
        if (i == j) y = li;
        else if (li == 0.0 || lj == 0.0) y = 0.0;
        else y = -a[i * LDM + j] * (li * lj) * (li * lj) / (li + lj);
        a[i * LDM + j] = y;
    }
    __syncthreads();
    // T = V Y over Y, then out = T V^T
    lds_gemm<false, false>(msz, v, a, a);
    lds_gemm<false, true>(msz, a, v, out);
}

// Sum over the 64 lanes of a wave by a fixed butterfly (every lane gets it).
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// s, c = sum of fp[w], cp[w] over w = sl, sl + step, ... < nwp, in that
// order.  The loads of B terms are issued together (indices past the end
// re-read the last term and add 0, which leaves the non-negative sums as they
// were), instead of one dependent load at a time.
template <int B>
__device__ __forceinline__ void slice_sum(const double* __restrict__ fp,
                                          const int* __restrict__ cp, int nwp, int sl, int step,
                                          double* s_out, int* c_out) {
    double s = 0.0;
    int c = 0;
    for (int w0 = sl; w0 < nwp; w0 += B * step) {
        double fv[B];
        int cv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int w = w0 + u * step;
            const int wc = w < nwp ? w : nwp - 1;
            fv[u] = fp[wc];
            cv[u] = cp[wc];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const bool in = w0 + u * step < nwp;
            s += in ? fv[u] : 0.0;
            c += in ? cv[u] : 0;
        }
    }
    *s_out = s;
    *c_out = c;
}

struct StopShared {
    double rot[kMaxM];
    double lam[kMaxM];
    double fj[kMaxM];
    int nj[kMaxM];
    int live[kMaxM];
    int dead[kMaxM];
    double dsc[kMaxM];  // original-form block L1: 1/||s_j|| (0 for a dead component)
    double fterm[kMaxM];  // component j's term of F
    int nlive, ndead, rankdef, stop;
};

// Retraction coefficients for the block forms with live set L and dead set D.
__device__ void block_coefficients(int m, double* coef, double* vprev, StopShared& ss,
                                   double* A0, double* A1, double* A2, Ctrl* ctrl) {
    const int t = threadIdx.x, nt = blockDim.x, mm = m * m;
    const double* GtG = coef + 2 * mm;
    const double* GtX = coef + 3 * mm;
    const double* XtX = coef + 4 * mm;
    double* Om = coef;
    double* Ps = coef + mm;
    const int nl = ss.nlive, nd = ss.ndead;
    for (int e = t; e < 2 * mm; e += nt) coef[e] = 0.0;
    // W_L = (G_L^T G_L)^{-1/2}
    const bool warm = (nd == 0) && ctrl->warm;
    for (int e = t; e < nl * nl; e += nt) {
        const int i = e / nl, j = e % nl;
        A0[i * LDM + j] = GtG[ss.live[i] * m + ss.live[j]];
        if (warm) A1[i * LDM + j] = vprev[i * m + j];
    }
    __syncthreads();
    if (warm) {
        // A0 <- V0^T M V0 with the previous pass's eigenvectors V0: the Gram matrix
        // changes little between passes, so this is nearly diagonal already
        lds_gemm<false, false>(nl, A0, A1, A2);
        lds_gemm<true, false>(nl, A1, A2, A0);
    }
    jacobi_eig(A0, A1, nl, ss.rot, warm);

    if (nd == 0) {
        for (int e = t; e < nl * nl; e += nt) {
            const int i = e / nl, j = e % nl;
            vprev[i * m + j] = A1[i * LDM + j];
        }
    }
    int rd1 = 0;
    inv_sqrt_from_eig(A0, A1, A2, nl, ss.lam, &ss.rankdef);

    rd1 = ss.rankdef;
    __syncthreads();
    // Omega[L,L] = W_L
    for (int e = t; e < nl * nl; e += nt) {
        const int i = e / nl, j = e % nl;
        Om[ss.live[i] * m + ss.live[j]] = A2[i * LDM + j];
    }
    if (nd > 0) {
        // C = W_L^T (G^T X)[L, D]   (nl x nd) -> A0
        __syncthreads();
        for (int e = t; e < nl * nd; e += nt) {
            const int a = e / nd, d = e % nd;
            double s = 0.0;
            for (int l = 0; l < nl; ++l) s += A2[l * LDM + a] * GtX[ss.live[l] * m + ss.dead[d]];
            A0[a * LDM + d] = s;
        }
        __syncthreads();
        // H^T H = (X^T X)[D,D] - C^T C -> A1
        for (int e = t; e < nd * nd; e += nt) {
            const int d1 = e / nd, d2 = e % nd;
            double s = XtX[ss.dead[d1] * m + ss.dead[d2]];
            for (int a = 0; a < nl; ++a) s -= A0[a * LDM + d1] * A0[a * LDM + d2];
            A1[d1 * LDM + d2] = s;
        }
        __syncthreads();
        // W_L C  (nl x nd) -> keep in Om scratch rows?  compute into A0 in place:
        // B = W_L C; needs W_L (A2) and C (A0): write B into Ps temporarily.
        for (int e = t; e < nl * nd; e += nt) {
            const int a = e / nd, d = e % nd;
            double s = 0.0;
            for (int l = 0; l < nl; ++l) s += A2[a * LDM + l] * A0[l * LDM + d];
            Ps[a * m + d] = s;  // temporary (nl x nd, leading dim m)
        }
        __syncthreads();
        // W_D = (H^T H)^{-1/2}: eig of A1 into (A1, A0), inverse root into A2
        for (int e = t; e < nd * nd; e += nt) {
            const int i = e / nd, j = e % nd;
            A0[i * LDM + j] = A1[i * LDM + j];
        }
        __syncthreads();
        jacobi_eig(A0, A1, nd, ss.rot);
        inv_sqrt_from_eig(A0, A1, A2, nd, ss.lam, &ss.rankdef);
        // Omega[L,D] = -(W_L C) W_D ; Psi[D,D] = W_D
        double* tmp = A0;  // nl x nd product
        for (int e = t; e < nl * nd; e += nt) {
            const int a = e / nd, d = e % nd;
            double s = 0.0;
            for (int k = 0; k < nd; ++k) s += Ps[a * m + k] * A2[k * LDM + d];
            tmp[a * LDM + d] = -s;
        }
        __syncthreads();
        for (int e = t; e < mm; e += nt) Ps[e] = 0.0;
        __syncthreads();
        for (int e = t; e < nl * nd; e += nt) {
            const int a = e / nd, d = e % nd;
            Om[ss.live[a] * m + ss.dead[d]] = tmp[a * LDM + d];
        }
        for (int e = t; e < nd * nd; e += nt) {
            const int i = e / nd, j = e % nd;
            Ps[ss.dead[i] * m + ss.dead[j]] = A2[i * LDM + j];
        }
        __syncthreads();
    }
    if (t == 0) {
        ctrl->ndead = nd;
        ctrl->warm = (nd == 0) ? 1 : 0;
        if (nd > 0 || rd1 || ss.rankdef) ctrl->degenerate_seen = 1;
    }
    __syncthreads();
}

// Objective of a pass, its trace entry and the stopping rule, by the whole
// workgroup: per-component terms f_j and support sizes from the fixed-order
// sums of the wave partials, F, and the rule (F = 0, the relative change
// below tol, or the last allowed pass).  Fills ss (terms, live and dead
// components, stop) and the control block; returns the stop flag.
// kGiven: fsum is always given (the branch that sums the partials is left out).
template <bool kGiven = false>
__device__ int stop_rule(int m, int nwp, const double* __restrict__ fpart,
                         const int* __restrict__ nnzpart, double* __restrict__ trace,
                         double* __restrict__ fcomp, int exact, Ctrl* __restrict__ ctrl,
                         StopShared& ss, const double* __restrict__ fsum = nullptr) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int k = ctrl->k;
    // the control fields the stopping rule needs, loaded up front so their
    // latency overlaps the sums
    const double last_F = ctrl->last_F, tol = ctrl->tol;
    const int max_iter = ctrl->max_iter, deg_seen = ctrl->degenerate_seen;

    // per-component objective and support size: summed already (fsum, by the
    // Gram-sum kernel), or here by tpc (a power of two <= 64) lanes of one
    // wave per component, each summing a strided slice, the slices combined by
    // a fixed butterfly (fixed order)
    if (kGiven || fsum) {
        for (int j = t; j < m; j += nt) {
            ss.fj[j] = fsum[j];
            ss.nj[j] = (int)fsum[m + j];
        }
    } else {
        int tpc = 64;
        while (tpc > 1 && tpc * m > nt) tpc >>= 1;
        for (int j0 = 0; j0 < m; j0 += nt / tpc) {
            const int j = j0 + t / tpc, sl = t % tpc;
            double s = 0.0;
            int c = 0;
            if (j < m) slice_sum<32>(fpart + (size_t)j * nwp, nnzpart + (size_t)j * nwp, nwp, sl, tpc,
                                 &s, &c);
            for (int o = tpc / 2; o >= 1; o >>= 1) {
                s += __shfl_xor(s, o, 64);
                c += __shfl_xor(c, o, 64);
            }
            if (sl == 0 && j < m) {
                ss.fj[j] = s;
                ss.nj[j] = c;
            }
        }
    }
    __syncthreads();
    // per-component terms in parallel (original form of block L1: ||s_j||)
    for (int j = t; j < m; j += nt) {
        const double fj = ss.fj[j];
        ss.fterm[j] = exact ? sqrt(fj) : fj;
        ss.dsc[j] = (exact && fj > 0.0) ? 1.0 / sqrt(fj) : 0.0;
        fcomp[j] = fj;
        reinterpret_cast<int64_t*>(fcomp + m)[j] = ss.nj[j];
    }
    __syncthreads();
    if (t == 0) {
        double F = 0.0;
        int nl = 0, nd = 0;
        for (int j = 0; j < m; ++j) {
            F += ss.fterm[j];
            if (ss.nj[j] > 0) ss.live[nl++] = j;
            else ss.dead[nd++] = j;
        }
        ss.nlive = nl;
        ss.ndead = nd;
        trace[k] = F;
        int stop = 0, status = GPSPCA_OK;
        int degenerate = deg_seen;
        if (!isfinite(F)) {
            stop = 1;
            status = GPSPCA_ENONFINITE;
        } else if (F == 0.0) {
            stop = 1;
            degenerate = 1;
            ctrl->degenerate_seen = 1;
        } else if (k >= 1 && fabs(F - last_F) < tol * fabs(last_F)) {
            stop = 1;
        } else if (k + 1 >= max_iter) {
            stop = 1;
            status = GPSPCA_MAXITER;
        }
        if (stop) {
            if (status >= 0 && degenerate) status = GPSPCA_DEGENERATE;
            ctrl->status = status;
            ctrl->done = 1;
            ctrl->n_iter = k + 1;
        }
        ctrl->last_F = F;
        ss.stop = stop;
    }
    __syncthreads();
    return ss.stop;
}

// m = 1: ||g||^2 as the sum of the ngram Gram partials (entry 0 of each
// 3-entry block; strided per-thread sums, a fixed butterfly in each wave, the
// waves in order), 1/||g|| into coef, and the check that it is finite.
// Returns 1/||g|| to every thread, or 0 when the pass failed.  red: at least
// blockDim.x / 64 doubles of LDS.
__device__ double unit_scale(const double* __restrict__ gram, int ngram,
                             double* __restrict__ coef, int k, Ctrl* __restrict__ ctrl,
                             double* red) {
    const int t = threadIdx.x, nt = blockDim.x;
    double sg = 0.0;
    for (int g = t; g < ngram; g += nt) sg += gram[(size_t)3 * g];
    sg = wave_sum_d(sg);
    if ((t & 63) == 0) red[t >> 6] = sg;
    __syncthreads();
    if (t == 0) {
        double g2 = 0.0;
        for (int u = 0; u < (nt + 63) / 64; ++u) g2 += red[u];
        coef[2] = g2;
        const double om = 1.0 / sqrt(g2);
        coef[0] = om;
        coef[1] = 0.0;
        ctrl->ndead = 0;
        const int bad = (!(g2 > 0.0) || !isfinite(om)) ? 1 : 0;
        if (bad) {
            ctrl->status = GPSPCA_ENONFINITE;
            ctrl->done = 1;
            ctrl->n_iter = k + 1;
        }
        red[0] = bad ? 0.0 : om;
    }
    __syncthreads();
    return red[0];
}

// One workgroup: objective, trace, stopping rule, retraction coefficients.
// m = 1: ||g||^2 is summed here from the ngram Gram partials (no k_gram_sum),
// and with Xn given the retraction x_{k+1} = g / ||g|| is written here too
// (rows < p, FP32), in place of a separate apply launch.
__global__ __launch_bounds__(1024) void k_stop(int m, int nwp, const double* __restrict__ fpart,
                       const int* __restrict__ nnzpart, double* __restrict__ vprev,
                       double* __restrict__ trace, double* __restrict__ coef,
                       double* __restrict__ fcomp, const double* __restrict__ gram, int ngram,
                       int exact, const double* __restrict__ g64, float* __restrict__ Xn, int p,
                       const double* __restrict__ fsum, Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ StopShared ss;
    __shared__ double red[1024];
    extern __shared__ double dyn[];
    double* A0 = dyn;
    // three matrices of m rows rounded up to even (jacobi_eig pads odd sizes)
    const int mr = m + (m & 1);
    double* A1 = dyn + (size_t)mr * LDM;
    double* A2 = dyn + (size_t)2 * mr * LDM;
    const int t = threadIdx.x, nt = blockDim.x;
    const int k = ctrl->k;
    if (stop_rule(m, nwp, fpart, nnzpart, trace, fcomp, exact, ctrl, ss, m > 1 ? fsum : nullptr))
        return;

    const int mm = m * m;
    if (m == 1) {
        const double om = unit_scale(gram, ngram, coef, k, ctrl, red);
        if (Xn && om != 0.0)
            for (int r = t; r < p; r += nt) Xn[r] = (float)(g64[r] * om);
    } else {
        if (exact) {
            // direction G D, D = Diag(1/||s_j||): G^T G <- D G^T G D, G^T X <- D G^T X
            for (int e = t; e < mm; e += nt) {
                const int a = e / m, b = e % m;
                coef[2 * mm + e] *= ss.dsc[a] * ss.dsc[b];
                coef[3 * mm + e] *= ss.dsc[a];
            }
            __syncthreads();
        }
        block_coefficients(m, coef, vprev, ss, A0, A1, A2, ctrl);
        if (exact) {
            // X_{k+1} = (G D) Omega + X_k Psi: row l of Omega takes 1/||s_l||
            __syncthreads();
            for (int e = t; e < mm; e += nt) coef[e] *= ss.dsc[e / m];
            __syncthreads();
        }
        // finiteness of the coefficients (every thread checks its share)
        int bad = 0;
        for (int e = t; e < 2 * mm; e += nt) bad |= isfinite(coef[e]) ? 0 : 1;
        if (__syncthreads_or(bad) && t == 0) {
            ctrl->status = GPSPCA_ENONFINITE;
            ctrl->done = 1;
            ctrl->n_iter = k + 1;
            ctrl->warm = 0;
        }
        __syncthreads();
    }
    if (t == 0 && !ctrl->done) {
        ctrl->k = k + 1;
        ctrl->nact = 0;   // the next pass counts its active columns afresh
    }
}

// Single unit (m = 1) with the retraction written here: stopping rule, ||g||^2
// from the Gram partials and x_{k+1} = g / ||g|| (rows < p, FP32).  Wave 0
// sums the objective and support-size partials (lane l the partials l, l + 64,
// ..., then a fixed butterfly) while waves 1.. load their rows of g (kX1Rows
// each: rows u, u + nt - 64, ... for u = t - 64), so that the latency of both
// overlaps; rows past kX1Rows * (nt - 64), if any, are read afterwards.
constexpr int kX1Rows = 22;   // 22 * 960 >= 20480, the largest p of the fused pass
__global__ __launch_bounds__(1024) void k_stop_x1(int nwp, const double* __restrict__ fpart,
                                                  const int* __restrict__ nnzpart,
                                                  double* __restrict__ trace,
                                                  double* __restrict__ coef,
                                                  double* __restrict__ fcomp,
                                                  const double* __restrict__ gram, int ngram,
                                                  int exact, const double* __restrict__ g64,
                                                  float* __restrict__ Xn, int p,
                                                  Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ StopShared ss;
    __shared__ double red[16];
    __shared__ double fs[2];
    const int t = threadIdx.x, nt = blockDim.x, lane = t & 63;
    const int u0 = t - 64, ust = nt - 64;
    double gx[kX1Rows];
    if (t < 64) {
        double sf;
        int sc;
        slice_sum<8>(fpart, nnzpart, nwp, lane, 64, &sf, &sc);
        for (int o = 32; o >= 1; o >>= 1) {
            sf += __shfl_xor(sf, o, 64);
            sc += __shfl_xor(sc, o, 64);
        }
        if (lane == 0) {
            fs[0] = sf;
            fs[1] = (double)sc;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kX1Rows; ++i) {
            const int r = u0 + i * ust;
            gx[i] = r < p ? g64[r] : 0.0;
        }
    }
    __syncthreads();
    const int k = ctrl->k;
    if (stop_rule<true>(1, nwp, fpart, nnzpart, trace, fcomp, exact, ctrl, ss, fs)) return;
    const double om = unit_scale(gram, ngram, coef, k, ctrl, red);
    if (om != 0.0) {
        if (t >= 64) {
#pragma unroll
            for (int i = 0; i < kX1Rows; ++i) {
                const int r = u0 + i * ust;
                if (r < p) Xn[r] = (float)(gx[i] * om);
            }
        }
        for (int r = kX1Rows * ust + t; r < p; r += nt) Xn[r] = (float)(g64[r] * om);
    }
    if (t == 0 && !ctrl->done) {
        ctrl->k = k + 1;
        ctrl->nact = 0;
    }
}

// m = 1 after the fused pass (one partial g per workgroup, every one written):
// g = the sum of the partials and the Gram partials of ||g||^2 in one launch.
// A workgroup owns kRm1Rows rows; slice sl (threads sl kRm1Rows .. + kRm1Rows
// - 1) of its kRm1Slices sums the contiguous range sl of the partials (all
// loads of a batch issued together), wave 0 adds the ranges in order, writes g
// (FP64) and the block's sum of g_r^2 (a fixed butterfly) as gram[3 * block].  Rows past p re-read row
// p - 1 and are dropped.
constexpr int kRm1Slices = 1024 / kRm1Rows, kRm1Batch = 16;
__global__ __launch_bounds__(1024) void k_reduce_m1(const float* __restrict__ gpart, int npart,
                                                    int ldx, int p, double* __restrict__ g64,
                                                    double* __restrict__ gram,
                                                    const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double part[kRm1Slices][kRm1Rows];
    const int t = threadIdx.x, rr = t % kRm1Rows, sl = t / kRm1Rows;
    const int r = blockIdx.x * kRm1Rows + rr;
    const int rc = r < p ? r : p - 1;
    const int c0 = (int)((int64_t)npart * sl / kRm1Slices);
    const int c1 = (int)((int64_t)npart * (sl + 1) / kRm1Slices);
    double s = 0.0;
    for (int c = c0; c < c1; c += kRm1Batch) {
        float v[kRm1Batch];
#pragma unroll
        for (int u = 0; u < kRm1Batch; ++u) {
            const int cu = c + u < c1 ? c + u : c1 - 1;
            v[u] = gpart[(size_t)cu * ldx + rc];
        }
#pragma unroll
        for (int u = 0; u < kRm1Batch; ++u) s += (c + u < c1) ? (double)v[u] : 0.0;
    }
    part[sl][rr] = s;
    __syncthreads();
    if (t < 64) {   // wave 0: lanes t < kRm1Rows finish the rows, the rest add 0
        const bool own = t < kRm1Rows && r < p;
        double g = 0.0;
        if (t < kRm1Rows) {
            g = part[0][rr];
#pragma unroll
            for (int u = 1; u < kRm1Slices; ++u) g += part[u][rr];
        }
        if (own) g64[r] = g;
        const double g2 = wave_sum_d(own ? g * g : 0.0);
        if (t == 0) gram[(size_t)3 * blockIdx.x] = g2;
    }
}

hipError_t launch_reduce_m1(const Plan& pl, const float* gpart, double* g64, double* gram,
                            const Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_m1, dim3((unsigned)((pl.p + kRm1Rows - 1) / kRm1Rows)), dim3(1024), 0, st,
                       gpart, pl.npart, pl.ldx, (int)pl.p, g64, gram, ctrl);
    return hipGetLastError();
}

hipError_t launch_stop(const Plan& pl, const double* fpart, const int* nnzpart,
                       const double* gram, double* trace, double* coef, double* fcomp,
                       double* vprev, const double* g64, float* Xn, double* fsum, Ctrl* ctrl,
                       hipStream_t st) {
    if (pl.m > 1) {
        hipError_t e = launch_gram_sum(pl, 3 * pl.m * pl.m, pl.gram_blocks, gram, coef, ctrl, st,
                                       fpart, nnzpart, fsum);
        if (e != hipSuccess) return e;
    }
    if (pl.m == 1 && Xn) {
        hipLaunchKernelGGL(k_stop_x1, dim3(1), dim3(1024), 0, st, pl.nwave_part, fpart, nnzpart,
                           trace, coef, fcomp, gram, pl.gram_blocks, pl.exact, g64, Xn,
                           (int)pl.p, ctrl);
        return hipGetLastError();
    }
    // threads: the Jacobi steps of m = 64 have 32 x 32 blocks plus 64 x 32 rotated pairs of V;
    // m = 1 needs no eigen-solver: one wave makes every barrier free
    const int threads = pl.m > 1 ? jacobi_threads(pl.m) : 64;
    const size_t shm = (pl.m > 1) ? (size_t)3 * (pl.m + (pl.m & 1)) * LDM * sizeof(double) : 0;
    static const bool lds_once = (set_lds_limit((const void*)k_stop), true);
    (void)lds_once;
    hipLaunchKernelGGL(k_stop, dim3(1), dim3(threads), shm, st, pl.m, pl.nwave_part, fpart,
                       nnzpart, vprev, trace, coef, fcomp, gram, pl.gram_blocks, pl.exact,
                       g64, nullptr, (int)pl.p, fsum, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gamma path: m independent single-unit problems (column j has its own gamma).
// Per column: objective trace, stopping rule, and the sphere retraction
// x_j <- g_j / ||g_j||; a column whose rule fired is frozen (Psi_jj = 1), so
// its x, and with it S, F and Z, stay those of its stopping pass.
__global__ __launch_bounds__(1024) void k_stop_path(int m, int nwp, const double* __restrict__ fpart,
                            const int* __restrict__ nnzpart, double* __restrict__ trace,
                            double* __restrict__ coef, double* __restrict__ fcomp,
                            PathState* __restrict__ ps, Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double red[1024];
    __shared__ int redi[1024];
    __shared__ double fj[kMaxM];
    __shared__ int nj[kMaxM];
    __shared__ int nfrozen;
    const int t = threadIdx.x, nt = blockDim.x, mm = m * m;
    const int k = ctrl->k;
    const int max_iter = ctrl->max_iter;
    const double tol = ctrl->tol;
    // per-column objective and support size: tpc threads per column, each
    // summing a strided slice, the slices added in order (fixed order)
    {
        const int tpc = nt / m >= 1 ? nt / m : 1;
        for (int j0 = 0; j0 < m; j0 += nt / tpc) {
            const int j = j0 + t / tpc, sl = t % tpc;
            double s = 0.0;
            int c = 0;
            if (j < m && t / tpc < nt / tpc)
                slice_sum<16>(fpart + (size_t)j * nwp, nnzpart + (size_t)j * nwp, nwp, sl, tpc, &s, &c);
            red[t] = s;
            redi[t] = c;
            __syncthreads();
            if (sl == 0 && j < m && t / tpc < nt / tpc) {
                double a = 0.0;
                int b = 0;
                for (int q = 0; q < tpc; ++q) {
                    a += red[t + q];
                    b += redi[t + q];
                }
                fj[j] = a;
                nj[j] = b;
            }
            __syncthreads();
        }
    }
    if (t == 0) nfrozen = 0;
    for (int e = t; e < 2 * mm; e += nt) coef[e] = 0.0;  // Omega, Psi (the summed Gram is at 2mm)
    __syncthreads();
    for (int j = t; j < m; j += nt) {
        const double F = fj[j];
        fcomp[j] = F;
        reinterpret_cast<int64_t*>(fcomp + m)[j] = nj[j];
        PathState st = ps[j];
        if (!st.frozen) {
            trace[(size_t)j * max_iter + k] = F;
            int stop = 0, status = GPSPCA_OK;
            if (!isfinite(F)) {
                stop = 1;
                status = GPSPCA_ENONFINITE;
            } else if (F == 0.0) {
                stop = 1;
                st.degenerate = 1;
            } else if (k >= 1 && fabs(F - st.last_F) < tol * fabs(st.last_F)) {
                stop = 1;
            } else if (k + 1 >= max_iter) {
                stop = 1;
                status = GPSPCA_MAXITER;
            }
            if (stop) {
                st.frozen = 1;
                st.n_iter = k + 1;
                st.status = (status >= 0 && st.degenerate) ? GPSPCA_DEGENERATE : status;
            }
            st.last_F = F;
            ps[j] = st;
        }
        const double g2 = coef[2 * mm + (size_t)j * m + j];
        if (st.frozen) {
            coef[mm + j * m + j] = 1.0;
            atomicAdd(&nfrozen, 1);
        } else {
            coef[j * m + j] = 1.0 / sqrt(g2);
        }
    }
    __syncthreads();
    if (t == 0) {
        if (nfrozen == m) {
            ctrl->done = 1;
            ctrl->n_iter = k + 1;
        } else {
            ctrl->ndead = nfrozen > 0 ? 1 : 0;
            ctrl->k = k + 1;
        }
        ctrl->last_F = 0.0;
        ctrl->nact = 0;   // the next pass counts its active columns afresh
    }
}

hipError_t launch_stop_path(const Plan& pl, const double* fpart, const int* nnzpart,
                            const double* gram, double* trace, double* coef, double* fcomp,
                            PathState* ps, Ctrl* ctrl, hipStream_t st) {
    hipError_t e = launch_gram_sum(pl, pl.m * pl.m, pl.gram_blocks, gram, coef, ctrl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stop_path, dim3(1), dim3(1024), 0, st, pl.m, pl.nwave_part, fpart,
                       nnzpart, trace, coef, fcomp, ps, ctrl);
    return hipGetLastError();
}

// X[:, j] <- X[:, 0] for 1 <= j < m (rows < p)
__global__ void k_bcast_col0(int m, int p, int ldx, float* __restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)(m - 1) * p) return;
    const int j = 1 + (int)(e / p), r = (int)(e % p);
    X[(size_t)j * ldx + r] = X[r];
}

hipError_t launch_bcast_col0(const Plan& pl, float* X, hipStream_t st) {
    if (pl.m < 2) return hipSuccess;
    const int64_t ne = (int64_t)(pl.m - 1) * pl.p;
    hipLaunchKernelGGL(k_bcast_col0, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, pl.m,
                       (int)pl.p, pl.ldx, X);
    return hipGetLastError();
}

// Column-wise normalization of a starting point (gamma path): Omega =
// diag(1/||x_j||); a zero column fails with GPSPCA_EINVAL.
__global__ void k_project_diag(int m, double* __restrict__ coef, Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    const int t = threadIdx.x, mm = m * m;
    for (int e = t; e < 2 * mm; e += blockDim.x) coef[e] = 0.0;
    __syncthreads();
    for (int j = t; j < m; j += blockDim.x) {
        const double g2 = coef[2 * mm + (size_t)j * m + j];
        const double om = 1.0 / sqrt(g2);
        coef[j * m + j] = om;
        if (!(g2 > 0.0) || !isfinite(om)) {
            ctrl->status = GPSPCA_EINVAL;
            ctrl->done = 1;
        }
    }
    if (t == 0) ctrl->ndead = 0;
}

hipError_t launch_project_diag(const Plan& pl, const double* gram, double* coef, Ctrl* ctrl,
                               hipStream_t st) {
    hipError_t e = launch_gram_sum(pl, pl.m * pl.m, pl.gram_grid, gram, coef, ctrl, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_project_diag, dim3(1), dim3(256), 0, st, pl.m, coef, ctrl);
    return hipGetLastError();
}

// Projection of a starting point onto the feasible set: Omega = (G^T G)^{-1/2}
// (or 1/||g||); a rank-deficient start fails with GPSPCA_EINVAL.
__global__ void k_project(int m, double* __restrict__ coef, Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ StopShared ss;
    extern __shared__ double dyn[];
    double* A0 = dyn;
    // three matrices of m rows rounded up to even (jacobi_eig pads odd sizes)
    const int mr = m + (m & 1);
    double* A1 = dyn + (size_t)mr * LDM;
    double* A2 = dyn + (size_t)2 * mr * LDM;
    const int t = threadIdx.x, nt = blockDim.x, mm = m * m;
    if (m == 1) {
        if (t == 0) {
            const double g2 = coef[2];
            coef[0] = 1.0 / sqrt(g2);
            coef[1] = 0.0;
            if (!(g2 > 0.0) || !isfinite(coef[0])) {
                ctrl->status = GPSPCA_EINVAL;
                ctrl->done = 1;
            }
        }
        return;
    }
    for (int e = t; e < mm; e += nt) {
        const int i = e / m, j = e % m;
        A0[i * LDM + j] = coef[2 * mm + e];
    }
    __syncthreads();
    jacobi_eig(A0, A1, m, ss.rot);
    inv_sqrt_from_eig(A0, A1, A2, m, ss.lam, &ss.rankdef);
    for (int e = t; e < mm; e += nt) {
        const int i = e / m, j = e % m;
        coef[e] = A2[i * LDM + j];
        coef[mm + e] = 0.0;
    }
    if (t == 0) {
        ctrl->ndead = 0;
        ctrl->warm = 0;
        if (ss.rankdef) {
            ctrl->status = GPSPCA_EINVAL;
            ctrl->done = 1;
        }
    }
}

hipError_t launch_project(const Plan& pl, const double* gram, double* coef, Ctrl* ctrl,
                          hipStream_t st) {
    hipError_t e = launch_gram_sum(pl, pl.m * pl.m, pl.gram_grid, gram, coef, ctrl, st);
    if (e != hipSuccess) return e;
    const int threads = jacobi_threads(pl.m);
    const size_t shm = (pl.m > 1) ? (size_t)3 * (pl.m + (pl.m & 1)) * LDM * sizeof(double) : 0;
    static const bool lds_once = (set_lds_limit((const void*)k_project), true);
    (void)lds_once;
    hipLaunchKernelGGL(k_project, dim3(1), dim3(threads), shm, st, pl.m, coef, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X_{k+1}[r, j] = sum_l G[r, l] Omega[l, j] + sum_l X_k[r, l] Psi[l, j]
// grid (row blocks of 256, columns j): one output element per thread.
__global__ __launch_bounds__(256) void k_apply(int m, int p, int ldx,
                                               const double* __restrict__ g64,
                                               const float* __restrict__ Xk,
                                               const double* __restrict__ coef,
                                               float* __restrict__ Xn,
                                               float* __restrict__ Xil, int diag,
                                               const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double om[kMaxM];
    __shared__ double ps[kMaxM];
    const int t = threadIdx.x, j = blockIdx.y, mm = m * m;
    const bool dead = ctrl->ndead > 0;
    for (int l = t; l < m; l += 256) {
        om[l] = coef[l * m + j];
        ps[l] = dead ? coef[mm + l * m + j] : 0.0;
    }
    __syncthreads();
    const int r = blockIdx.x * 256 + t;
    if (r >= p) return;
    double acc = 0.0;
    int l = diag ? m : 0;  // gamma path: Omega and Psi are diagonal
    if (diag) {
        acc = g64[(size_t)j * p + r] * om[j];
        if (dead) acc += (double)Xk[(size_t)j * ldx + r] * ps[j];
    }
    for (; l + 4 <= m; l += 4) {  // in order of l, 4 loads issued together
        double gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) gv[u] = g64[(size_t)(l + u) * p + r];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += gv[u] * om[l + u];
    }
    for (; l < m; ++l) acc += g64[(size_t)l * p + r] * om[l];
    if (dead && !diag)
        for (int l = 0; l < m; ++l) acc += (double)Xk[(size_t)l * ldx + r] * ps[l];
    Xn[(size_t)j * ldx + r] = (float)acc;
    if (Xil)
        Xil[((size_t)((j >> 4) * (ldx >> 2) + (r >> 2)) * 16 + (j & 15)) * 4 + (r & 3)] = (float)acc;
}

// The same for m > 16 (full Omega and Psi): grid (row blocks of 256, groups of
// 16 components); each thread reads its row of G once and keeps 16 outputs,
// summing over l in the same order as k_apply (bitwise the same result), so G
// is read m / 16 instead of m times.
__global__ __launch_bounds__(256) void k_apply16(int m, int p, int ldx,
                                                 const double* __restrict__ g64,
                                                 const float* __restrict__ Xk,
                                                 const double* __restrict__ coef,
                                                 float* __restrict__ Xn, float* __restrict__ Xil,
                                                 const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double om[kMaxM][16];
    __shared__ double ps[kMaxM][16];
    const int t = threadIdx.x, jb = blockIdx.y * 16, mm = m * m;
    const int nj = (m - jb < 16) ? m - jb : 16;
    const bool dead = ctrl->ndead > 0;
    for (int e = t; e < m * 16; e += 256) {
        const int l = e >> 4, jj = e & 15;
        const int j = jb + (jj < nj ? jj : nj - 1);
        om[l][jj] = coef[l * m + j];
        ps[l][jj] = dead ? coef[mm + l * m + j] : 0.0;
    }
    __syncthreads();
    const int r = blockIdx.x * 256 + t;
    if (r >= p) return;
    double acc[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
    int l = 0;
    for (; l + 4 <= m; l += 4) {  // 4 loads issued together
        double gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) gv[u] = g64[(size_t)(l + u) * p + r];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] += gv[u] * om[l + u][jj];
    }
    for (; l < m; ++l) {
        const double gv = g64[(size_t)l * p + r];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] += gv * om[l][jj];
    }
    if (dead)
        for (int l2 = 0; l2 < m; ++l2) {
            const double xv = (double)Xk[(size_t)l2 * ldx + r];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] += xv * ps[l2][jj];
        }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        if (jj >= nj) break;
        const int j = jb + jj;
        const float v = (float)acc[jj];
        Xn[(size_t)j * ldx + r] = v;
        if (Xil)
            Xil[((size_t)((j >> 4) * (ldx >> 2) + (r >> 2)) * 16 + (j & 15)) * 4 + (r & 3)] = v;
    }
}

hipError_t launch_apply(const Plan& pl, const double* g64, const float* Xk, const double* coef,
                        float* Xn, float* Xil_n, const Ctrl* ctrl, hipStream_t st) {
    const int p = (int)pl.p;
    if (pl.m > 16 && !pl.path) {
        hipLaunchKernelGGL(k_apply16, dim3((p + 255) / 256, (pl.m + 15) / 16), dim3(256), 0, st,
                           pl.m, p, pl.ldx, g64, Xk, coef, Xn, Xil_n, ctrl);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_apply, dim3((p + 255) / 256, pl.m), dim3(256), 0, st, pl.m, p, pl.ldx,
                       g64, Xk, coef, Xn, Xil_n, pl.path, ctrl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deflated single-unit components.  P = I - Q Q^T with Q (p x k, leading dim
// p, FP64) the earlier components.
//
// k_deflate: out = P x / ||P x|| in FP64 from FP64 x, to FP32; one workgroup
// of 1024 threads.  Every sum is a fixed-order butterfly
// within each wave followed by the 16 wave sums added in wave order, eight dot
// products per barrier.  P x = 0 gives 0 (the next pass then has F = 0 and
// stops).  scratch == x is allowed: each thread reads and writes only its
// own rows.

__global__ __launch_bounds__(1024) void k_deflate(int p, int k, const double* __restrict__ Q,
                                                  const double* x, float* __restrict__ out,
                                                  double* scratch,
                                                  const Ctrl* __restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    constexpr int NW = 16;
    __shared__ double wpart[8][NW];
    __shared__ double c[kMaxM + 1];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int j0 = 0; j0 < k; j0 += 8) {
        const int nj = (k - j0 < 8) ? k - j0 : 8;
        double d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = 0.0;
        // basis vectors past the last re-read vector j0 + nj - 1 (a valid
        // address) and are dropped by a select: the 8 loads are issued together
        size_t qo[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) qo[u] = (size_t)(j0 + (u < nj ? u : nj - 1)) * p;
        for (int r = t; r < p; r += 1024) {
            const double xr = x[r];
            double q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) q[u] = Q[qo[u] + r];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] += (u < nj) ? q[u] * xr : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double v = wave_sum_d(d[u]);
            if (lane == 0) wpart[u][w] = v;
        }
        __syncthreads();
        if (t < nj) {
            double v = 0.0;
            for (int i = 0; i < NW; ++i) v += wpart[t][i];
            c[j0 + t] = v;
        }
        __syncthreads();
    }
    double s2 = 0.0;
    for (int r = t; r < p; r += 1024) {
        double y = x[r];
        int j = 0;
        for (; j + 4 <= k; j += 4) {
            double q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = Q[(size_t)(j + u) * p + r];
#pragma unroll
            for (int u = 0; u < 4; ++u) y -= q[u] * c[j + u];
        }
        for (; j < k; ++j) y -= Q[(size_t)j * p + r] * c[j];
        scratch[r] = y;
        s2 += y * y;
    }
    s2 = wave_sum_d(s2);
    if (lane == 0) wpart[0][w] = s2;
    __syncthreads();
    if (t == 0) {
        double v = 0.0;
        for (int i = 0; i < NW; ++i) v += wpart[0][i];
        c[kMaxM] = v;
    }
    __syncthreads();
    const double nrm2 = c[kMaxM];
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    for (int r = t; r < p; r += 1024) out[r] = (float)(scratch[r] * inv);
}

hipError_t launch_deflate(int p, int k, const double* Q, const double* x, float* out,
                          double* scratch, const Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL(k_deflate, dim3(1), dim3(1024), 0, st, p, k, Q, x, out, scratch, ctrl);
    return hipGetLastError();
}

// k_defl_norms: ||P a_i|| = sqrt(||a_i||^2 - sum_j (q_j^T a_i)^2) in FP64 for
// every column of the FP32 matrix (one wave per column at a time; the column
// is read k + 1 times, from cache after the first): the default start of a
// deflated component.  Each lane sums its rows lane, lane + 64, ... in order;
// the loads of 8 such rows are issued together (rows past p re-read row p - 1
// and add 0), instead of one dependent load per row.
__global__ __launch_bounds__(256) void k_defl_norms(const float* __restrict__ A, int64_t lda,
                                                    int p, int64_t n, int k,
                                                    const double* __restrict__ Q,
                                                    double* __restrict__ norms) {
    constexpr int U = 8;
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += nw) {
        const float* a = A + i * lda;
        double ss = 0.0;
        for (int r0 = lane; r0 < p; r0 += 64 * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = r0 + 64 * u;
                v[u] = a[r < p ? r : p - 1];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) ss += (r0 + 64 * u < p) ? (double)v[u] * v[u] : 0.0;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
        double dd = 0.0;
        for (int j = 0; j < k; ++j) {
            const double* q = Q + (size_t)j * p;
            double d = 0.0;
            for (int r0 = lane; r0 < p; r0 += 64 * U) {
                float v[U];
                double qv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int r = r0 + 64 * u;
                    const int rc = r < p ? r : p - 1;
                    v[u] = a[rc];
                    qv[u] = q[rc];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) d += (r0 + 64 * u < p) ? qv[u] * v[u] : 0.0;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
            dd += d * d;
        }
        if (lane == 0) norms[i] = sqrt(fmax(ss - dd, 0.0));
    }
}

hipError_t launch_defl_norms(const float* A, int64_t lda, int p, int64_t n, int k,
                             const double* Q, double* norms, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_defl_norms, dim3(grid), dim3(256), 0, st, A, lda, p, n, k, Q, norms);
    return hipGetLastError();
}

// Q[:, k] = x (FP32 -> FP64)
__global__ void k_append_basis(int p, const float* __restrict__ x, double* __restrict__ q) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r < p) q[r] = (double)x[r];
}

hipError_t launch_append_basis(int p, const float* x, double* q, hipStream_t st) {
    hipLaunchKernelGGL(k_append_basis, dim3((p + 255) / 256), dim3(256), 0, st, p, x, q);
    return hipGetLastError();
}

// One thread per (block, quad, component): a 16-byte vector of 4 rows.
__global__ __launch_bounds__(256) void k_x_interleave(int mpad, int ldx,
                                                      const float* __restrict__ X,
                                                      float* __restrict__ Xil) {
    const int nq = ldx >> 2;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)nq * mpad) return;
    const int c = (int)(e % 16);
    const int64_t bq = e / 16;             // b * nq + q
    const int q = (int)(bq % nq), b = (int)(bq / nq);
    const float4 v = *reinterpret_cast<const float4*>(X + (size_t)(16 * b + c) * ldx + 4 * q);
    *reinterpret_cast<float4*>(Xil + (size_t)e * 4) = v;
}

hipError_t launch_x_interleave(const Plan& pl, const float* X, float* Xil, hipStream_t st) {
    const int64_t ne = (int64_t)(pl.ldx / 4) * pl.mpad;
    hipLaunchKernelGGL(k_x_interleave, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st,
                       pl.mpad, pl.ldx, X, Xil);
    return hipGetLastError();
}

// g64[j*p + r] = X0[j*ldx0 + r]
__global__ void k_load_g64(int m, int p, const float* __restrict__ X0, int ldx0,
                           double* __restrict__ g64) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)m * p) return;
    const int j = (int)(e / p), r = (int)(e % p);
    g64[e] = (double)X0[(size_t)j * ldx0 + r];
}

hipError_t launch_load_g64(const Plan& pl, const float* X0, int ldx0, double* g64,
                           hipStream_t st) {
    const int64_t ne = (int64_t)pl.m * pl.p;
    hipLaunchKernelGGL(k_load_g64, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, pl.m,
                       (int)pl.p, X0, ldx0, g64);
    return hipGetLastError();
}

}  // namespace gpspca
