// Reduced-precision storage of A on gfx950: the quantizer and the correlation
// kernel of the bfloat16 / e4m3fn path.
//
// Storage (an extension of the paper's method, which stores A in full
// precision): bfloat16 codes with scale 1, or e4m3fn codes with the per-column
// scale max_r |a_ri| / 448.  The correlation of a quantized column is
// scale_i * sum_r value(q_ri) x_rj, accumulated in FP32.
//
// k_corr_q streams the codes through LDS exactly like the FP32 matrix-core
// kernel (one wave per workgroup owning whole tiles of 16 columns, chunks of up
// to 64 columns, 8 swizzled 16-byte slots per column per stage, direct
// global->LDS DMA), but each slot now holds
// 8 (bfloat16) or 16 (e4m3) rows, and the products run on the bfloat16 matrix
// cores (v_mfma_f32_16x16x32_bf16):
//   - A codes are bfloat16 operands as loaded (e4m3 codes are widened to
//     bfloat16, which holds every e4m3 value exactly);
//   - X (FP32) is split as x = hi + mid + lo with three bfloat16 parts, so
//     the three products reproduce x to about 2^-24 relative: the dot product
//     keeps FP32 accuracy although A moves 2 or 1 bytes per element;
//   - the contraction index is permuted consistently on both operands: lane
//     group g of a 32-row step takes 8 consecutive rows of its slot.
#include "storage.h"

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

namespace gpspca {

typedef float f4q __attribute__((ext_vector_type(4)));
typedef __bf16 bf8q __attribute__((ext_vector_type(8)));
typedef uint32_t u4q __attribute__((ext_vector_type(4)));

namespace {

// --------------------------------------------------------------- quantizer
// bfloat16, round to nearest even on the FP32 bit pattern (A is finite).
__device__ __forceinline__ uint32_t bf16_rne(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// e4m3fn, round to nearest even, saturating at +-448.  Normal results: the
// FP32 exponent is rebiased (127 -> 7) and the 20 dropped mantissa bits are
// rounded on the bit pattern (a carry moves into the exponent field);
// subnormal results (|v| < 2^-6) are multiples of 2^-9.
__device__ __forceinline__ uint32_t e4m3_rne(float v) {
    const uint32_t u = __float_as_uint(v);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t mag = u & 0x7FFFFFFFu;
    uint32_t code;
    if (mag >= 0x43E00000u) {                 // |v| >= 448
        code = 0x7Eu;
    } else if (mag >= 0x3C800000u) {          // |v| >= 2^-6
        uint32_t x = mag - (120u << 23);
        x += 0x7FFFFu + ((x >> 20) & 1u);
        code = x >> 20;
        code = code < 0x7Eu ? code : 0x7Eu;
    } else {
        code = (uint32_t)__builtin_rintf(__uint_as_float(mag) * 512.0f);
    }
    return sign | code;
}

template <int TO>
__global__ __launch_bounds__(256) void k_quantize(const float* __restrict__ A, int64_t lda,
                                                  int p, int64_t n, void* __restrict__ out,
                                                  int64_t ldq, float* __restrict__ scale) {
    const int lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= n) return;
    const float* a = A + col * lda;
    if constexpr (TO == kStBF16) {
        uint16_t* q = static_cast<uint16_t*>(out) + col * ldq;
        for (int r = lane; r < p; r += 64) q[r] = (uint16_t)bf16_rne(a[r]);
        if (scale && lane == 0) scale[col] = 1.0f;
    } else {
        float mx = 0.f;
        for (int r = lane; r < p; r += 64) mx = fmaxf(mx, fabsf(a[r]));
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        const float sc = mx > 0.f ? mx / 448.0f : 1.0f;
        uint8_t* q = static_cast<uint8_t*>(out) + col * ldq;
        for (int r = lane; r < p; r += 64) q[r] = (uint8_t)e4m3_rne(a[r] / sc);
        if (lane == 0) scale[col] = sc;
    }
}

// ------------------------------------------------------- correlation kernel

__device__ __forceinline__ uint32_t q_slot(int c, int s) {
    return (uint32_t)(16 * (c * 8 + (s ^ ((c >> 1) & 7))));
}

template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void wait_lgkm() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void tie(f4q& v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ f4q lds16(uint32_t addr) {
    f4q v;
    asm volatile("ds_read_b128 %0, %1" : "=v"(v) : "v"(addr) : "memory");
    return v;
}

__device__ __forceinline__ void dma(const void* g, uint32_t lds) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                     (void __attribute__((address_space(3)))*)(uintptr_t)lds, 16,
                                     0, 0);
}

// Upper halves of two FP32 words packed as two bfloat16 (exact for values that
// are bfloat16 numbers).
__device__ __forceinline__ uint32_t pack_hi(float lo, float hi) {
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

// 8 e4m3 codes (two words) -> 8 bfloat16 operands.
__device__ __forceinline__ bf8q widen8(uint32_t w0, uint32_t w1) {
    const qf2 a = e4m3_pair(w0, false), b = e4m3_pair(w0, true);
    const qf2 c = e4m3_pair(w1, false), d = e4m3_pair(w1, true);
    u4q r = u4q{pack_hi(a.x, a.y), pack_hi(b.x, b.y), pack_hi(c.x, c.y), pack_hi(d.x, d.y)};
    return __builtin_bit_cast(bf8q, r);
}

// x = hi + mid + lo (each part bfloat16, rounded to nearest).
__device__ __forceinline__ void split3(const float (&x)[8], bf8q& hi, bf8q& mid, bf8q& lo) {
    float r[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        hi[e] = (__bf16)x[e];
        r[e] = x[e] - (float)hi[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        mid[e] = (__bf16)r[e];
        r[e] = r[e] - (float)mid[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) lo[e] = (__bf16)r[e];
}

__device__ __forceinline__ bool thresh_q(bool l0, double mu, double gamma, float y, float& s,
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

}  // namespace

// One chunk of NT tiles of 16 columns (NT <= 4) starting at column c0 (see
// k_corr_q).  Columns at or past cend are clamped to cend - 1 and dropped.
template <int NT, int ST, int J, int STAGES, int TMAX>
__device__ __forceinline__ void q_chunk(const PassParams& pp, int64_t c0, int64_t cend,
                                        uint32_t lbase, const float* const* xcol,
                                        const float* __restrict__ Xil, double* f_acc,
                                        int* nnz_acc, float* __restrict__ S,
                                        uint8_t* __restrict__ act) {
    int nact_l = 0;   // active columns written by this lane
    constexpr int ES = (ST == kStBF16) ? 2 : 1;     // bytes per element
    constexpr int EPS = 16 / ES;                     // rows per 16-byte slot
    constexpr int XQ = 2 * EPS;                      // X row quads per stage (8 slots)
    constexpr int XDMA = XQ / 4;                     // X DMA instructions per block
    constexpr int XBlk = XQ * 16 * 16;               // X bytes per component block
    constexpr int AStage = 16 * TMAX * 8 * 16;       // A bytes per stage: TMAX tiles x 8 slots
    constexpr int StageBytes = AStage + J * XBlk;
    constexpr int ADMA = 2 * NT;                     // A DMA instructions (8 columns each)
    constexpr int PER = ADMA + J * XDMA;
    constexpr int G8 = EPS / 8;                      // 8-row operand groups per slot
    const int lane = threadIdx.x;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nsf = p / EPS;                 // full slots per column
    const int nst = (nsf + 7) / 8;           // stages
    const int rows_main = nsf * EPS;
    const int nxq = nsf * (EPS / 4);         // X row quads covered by full slots
    const int nqx = pp.ldx >> 2;             // quads of the X buffers; the last is zero
    const bool l0 = pp.l0 != 0;
    const uint8_t* Ab = (ST == kStBF16) ? reinterpret_cast<const uint8_t*>(pp.Abf) : pp.Af8;
    const int64_t colbytes = pp.lda * ES;

    const uint8_t* acol[ADMA];
    int aslot[ADMA];
#pragma unroll
    for (int i = 0; i < ADMA; ++i) {
        const int L = 64 * i + lane;
        const int cl = L >> 3;
        aslot[i] = (L & 7) ^ ((cl >> 1) & 7);
        int64_t col = c0 + cl;
        col = (col < cend) ? col : cend - 1;
        acol[i] = Ab + col * colbytes;
    }
    auto issue = [&](int st) {
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
#pragma unroll
        for (int i = 0; i < ADMA; ++i) {
            int sl = 8 * st + aslot[i];
            sl = (sl < nsf) ? sl : nsf - 1;
            dma(acol[i] + 16 * sl, sb + 1024 * i);
        }
#pragma unroll
        for (int jb = 0; jb < J; ++jb)
#pragma unroll
            for (int i = 0; i < XDMA; ++i) {
                int q = XQ * st + 4 * i + lk;
                q = (q < nxq) ? q : nqx - 1;
                dma(Xil + ((size_t)(jb * nqx + q) * 16 + lj) * 4,
                    sb + AStage + XBlk * jb + 1024 * i);
            }
    };

    f4q acc[NT][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4q{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
        if (s < nst) issue(s);

    for (int st = 0; st < nst; ++st) {
        if (st + STAGES - 1 < nst) issue(st + STAGES - 1);
        const int ahead = (nst - 1 - st < STAGES - 1) ? nst - 1 - st : STAGES - 1;
        if constexpr (STAGES >= 3) {
            if (ahead >= 2) wait_vm<2 * PER>();
            else if (ahead == 1) wait_vm<PER>();
            else wait_vm<0>();
        } else {
            if (ahead >= 1) wait_vm<PER>();
            else wait_vm<0>();
        }
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int slot = 4 * h + lk;
            f4q araw[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) araw[t] = lds16(sb + q_slot(16 * t + lj, slot));
            f4q xr[J][EPS / 4];
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
#pragma unroll
                for (int u = 0; u < EPS / 4; ++u)
                    xr[jb][u] = lds16(sb + AStage + XBlk * jb +
                                      16u * (uint32_t)(((EPS / 4) * slot + u) * 16 + lj));
            wait_lgkm();
#pragma unroll
            for (int t = 0; t < NT; ++t) tie(araw[t]);
#pragma unroll
            for (int jb = 0; jb < J; ++jb)
#pragma unroll
                for (int u = 0; u < EPS / 4; ++u) tie(xr[jb][u]);
#pragma unroll
            for (int g = 0; g < G8; ++g) {
                bf8q xh[J], xm[J], xl[J];
#pragma unroll
                for (int jb = 0; jb < J; ++jb) {
                    float xv[8];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        xv[e] = xr[jb][2 * g][e];
                        xv[4 + e] = xr[jb][2 * g + 1][e];
                    }
                    split3(xv, xh[jb], xm[jb], xl[jb]);
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    bf8q aop;
                    if constexpr (ST == kStBF16) {
                        aop = __builtin_bit_cast(bf8q, araw[t]);
                    } else {
                        const u4q wv = __builtin_bit_cast(u4q, araw[t]);
                        aop = widen8(wv[2 * g], wv[2 * g + 1]);
                    }
#pragma unroll
                    for (int jb = 0; jb < J; ++jb) {
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xh[jb], acc[t][jb], 0, 0, 0);
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xm[jb], acc[t][jb], 0, 0, 0);
                        acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xl[jb], acc[t][jb], 0, 0, 0);
                    }
                }
            }
        }
    }

    // ragged tail rows rows_main .. p-1 (fewer than one slot), FP32 FMA
    if (rows_main < p) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t col = c0 + 16 * t + 4 * lk + v;
                col = (col < cend) ? col : cend - 1;
                const uint8_t* ac = Ab + col * colbytes;
                for (int r = rows_main; r < p; ++r) {
                    const float a = (ST == kStBF16)
                                        ? bf16_value(reinterpret_cast<const uint16_t*>(ac)[r])
                                        : e4m3_value(ac[r]);
#pragma unroll
                    for (int jb = 0; jb < J; ++jb)
                        acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                }
            }
    }

    // scale, threshold, S, activity flags
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + 16 * t + 4 * lk + v;
            const bool cvalid = col < cend;
            const float sc = cvalid ? column_scale(pp, col) : 1.0f;
            bool any = false;
#pragma unroll
            for (int jb = 0; jb < J; ++jb) {
                const int comp = 16 * jb + lj;
                if (cvalid && comp < m) {
                    float s;
                    double fv;
                    const bool a = thresh_q(l0, pp.mu[comp], pp.gam[comp], sc * acc[t][jb][v],
                                            s, fv);
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

// ST: kStBF16 | kStF8;  J: component blocks of 16;  STAGES: stages in flight.
// Work partition as in k_corr_mfma: whole tiles of 16 columns per wave.
template <int ST, int J, int STAGES, int TMAX = 4>
__global__ __launch_bounds__(64) void k_corr_q(PassParams pp, const float* __restrict__ X,
                                               const float* __restrict__ Xil,
                                               float* __restrict__ S, uint8_t* __restrict__ act,
                                               double* __restrict__ fpart,
                                               int* __restrict__ nnzpart,
                                               const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int EPS = (ST == kStBF16) ? 8 : 16;
    constexpr int XBlk = 2 * EPS * 16 * 16;
    constexpr int StageBytes = 16 * TMAX * 8 * 16 + J * XBlk;
    __shared__ __attribute__((aligned(16))) uint8_t lds[STAGES * StageBytes];
    const uint32_t lbase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)lds;

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

    // chunks of up to TMAX tiles; the chunk code is specialized per tile count
    for (int64_t c0 = cbeg; c0 < cend; c0 += 16 * TMAX) {
        const int64_t left = cend - c0;
        const int nt = left >= 16 * TMAX ? TMAX : (int)((left + 15) / 16);
#define GPSPCA_QC(NT) q_chunk<NT, ST, J, STAGES, TMAX>(pp, c0, cend, lbase, xcol, Xil, f_acc, nnz_acc, S, act)
        if constexpr (TMAX == 8) {
            switch (nt) {
                case 8: GPSPCA_QC(8); break;
                case 7: GPSPCA_QC(7); break;
                case 6: GPSPCA_QC(6); break;
                case 5: GPSPCA_QC(5); break;
                case 4: GPSPCA_QC(4); break;
                case 3: GPSPCA_QC(3); break;
                case 2: GPSPCA_QC(2); break;
                default: GPSPCA_QC(1); break;
            }
        } else {
            switch (nt) {
                case 4: GPSPCA_QC(4); break;
                case 3: GPSPCA_QC(3); break;
                case 2: GPSPCA_QC(2); break;
                default: GPSPCA_QC(1); break;
            }
        }
#undef GPSPCA_QC
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

// ---------------------------------------------------------------------------
// k_corr_qw: k_corr_q with four waves per workgroup that stream the same row
// stages in lockstep over their own columns and share each stage of X in
// LDS.  X stays FP32 (its three bfloat16 parts are made at the operand), so
// at 32 components a wave alone stages twice as many X bytes as e4m3 codes;
// shared, each wave issues a quarter of the X instructions.  The workgroup
// owns whole tiles of 16 columns; in each round every wave takes its share
// (up to TMAX tiles) of the round's tiles, and every wave executes the same
// barriers, including a wave with no tiles in a round (it still moves its
// share of X).
//   stage: per wave TMAX tiles x 8 slots of A (2 KB per tile), then X (XBlk
//   per component block); per stage, wave w waits for its own DMAs, the
//   barrier makes everyone's visible and frees the slot read in the last
//   stage, then w issues its DMAs for the stage STAGES - 1 ahead.
// ---------------------------------------------------------------------------
template <int NT, int ST, int J, int STAGES, int TMAX>
__device__ __forceinline__ void qw_round(const PassParams& pp, int64_t c0, int64_t cend,
                                         uint32_t lbase, int wv, const float* const* xcol,
                                         const float* __restrict__ Xil, double* f_acc,
                                         int* nnz_acc, float* __restrict__ S,
                                         uint8_t* __restrict__ act) {
    int nact_l = 0;   // active columns written by this lane
    constexpr int ES = (ST == kStBF16) ? 2 : 1;     // bytes per element
    constexpr int EPS = 16 / ES;                     // rows per 16-byte slot
    constexpr int XQ = 2 * EPS;                      // X row quads per stage (8 slots)
    constexpr int XDMA = XQ / 4;                     // X DMA instructions per block
    constexpr int XBlk = XQ * 16 * 16;               // X bytes per component block
    constexpr int AW = TMAX * 2048;                  // A bytes per wave per stage
    constexpr int StageBytes = 4 * AW + J * XBlk;
    constexpr int ADMA = 2 * NT;                     // A DMA instructions (8 columns each)
    constexpr int XW = J * XDMA / 4;                 // X DMA instructions per wave
    static_assert((J * XDMA) % 4 == 0, "X instructions split over four waves");
    constexpr int PER = ADMA + XW;
    constexpr int G8 = EPS / 8;                      // 8-row operand groups per slot
    const int lane = threadIdx.x & 63;
    const int lj = lane & 15, lk = lane >> 4;
    const int p = pp.p, m = pp.m;
    const int nsf = p / EPS;                 // full slots per column
    const int nst = (nsf + 7) / 8;           // stages
    const int rows_main = nsf * EPS;
    const int nxq = nsf * (EPS / 4);         // X row quads covered by full slots
    const int nqx = pp.ldx >> 2;             // quads of the X buffers; the last is zero
    const bool l0 = pp.l0 != 0;
    const uint8_t* Ab = (ST == kStBF16) ? reinterpret_cast<const uint8_t*>(pp.Abf) : pp.Af8;
    const int64_t colbytes = pp.lda * ES;

    const uint8_t* acol[ADMA > 0 ? ADMA : 1];
    int aslot[ADMA > 0 ? ADMA : 1];
#pragma unroll
    for (int i = 0; i < ADMA; ++i) {
        const int L = 64 * i + lane;
        const int cl = L >> 3;
        aslot[i] = (L & 7) ^ ((cl >> 1) & 7);
        int64_t col = c0 + cl;
        col = (col < cend) ? col : cend - 1;
        acol[i] = Ab + col * colbytes;
    }
    auto issue = [&](int st) {
        const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
#pragma unroll
        for (int i = 0; i < ADMA; ++i) {
            int sl = 8 * st + aslot[i];
            sl = (sl < nsf) ? sl : nsf - 1;
            dma(acol[i] + 16 * sl, sb + wv * AW + 1024 * i);
        }
#pragma unroll
        for (int u = 0; u < XW; ++u) {
            const int idx = wv + 4 * u;          // instruction idx = XDMA jb + i
            const int jb = idx / XDMA, i = idx % XDMA;
            int q = XQ * st + 4 * i + lk;
            q = (q < nxq) ? q : nqx - 1;
            dma(Xil + ((size_t)(jb * nqx + q) * 16 + lj) * 4, sb + 4 * AW + XBlk * jb + 1024 * i);
        }
    };

    f4q acc[NT > 0 ? NT : 1][J];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int jb = 0; jb < J; ++jb) acc[t][jb] = f4q{0.f, 0.f, 0.f, 0.f};

    // the previous round's last stage may still be read by other waves
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < STAGES - 1; ++s2)
        if (s2 < nst) issue(s2);

    for (int st = 0; st < nst; ++st) {
        // own DMAs of stage st done: later stages issued so far are st+1 .. st+STAGES-2
        const int later = (nst - 1 - st < STAGES - 2) ? nst - 1 - st : STAGES - 2;
        if constexpr (STAGES >= 3) {
            if (later >= 1) wait_vm<PER>();
            else wait_vm<0>();
        } else {
            (void)later;
            wait_vm<0>();
        }
        __syncthreads();
        if (st + STAGES - 1 < nst) issue(st + STAGES - 1);
        if constexpr (NT > 0) {
            const uint32_t sb = lbase + (uint32_t)((st % STAGES) * StageBytes);
            const uint32_t sa = sb + wv * AW, sx = sb + 4 * AW;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int slot = 4 * h + lk;
                f4q araw[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) araw[t] = lds16(sa + q_slot(16 * t + lj, slot));
                f4q xr[J][EPS / 4];
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
#pragma unroll
                    for (int u = 0; u < EPS / 4; ++u)
                        xr[jb][u] = lds16(sx + XBlk * jb +
                                          16u * (uint32_t)(((EPS / 4) * slot + u) * 16 + lj));
                wait_lgkm();
#pragma unroll
                for (int t = 0; t < NT; ++t) tie(araw[t]);
#pragma unroll
                for (int jb = 0; jb < J; ++jb)
#pragma unroll
                    for (int u = 0; u < EPS / 4; ++u) tie(xr[jb][u]);
#pragma unroll
                for (int g = 0; g < G8; ++g) {
                    bf8q xh[J], xm[J], xl[J];
#pragma unroll
                    for (int jb = 0; jb < J; ++jb) {
                        float xv[8];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            xv[e] = xr[jb][2 * g][e];
                            xv[4 + e] = xr[jb][2 * g + 1][e];
                        }
                        split3(xv, xh[jb], xm[jb], xl[jb]);
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        bf8q aop;
                        if constexpr (ST == kStBF16) {
                            aop = __builtin_bit_cast(bf8q, araw[t]);
                        } else {
                            const u4q wv4 = __builtin_bit_cast(u4q, araw[t]);
                            aop = widen8(wv4[2 * g], wv4[2 * g + 1]);
                        }
#pragma unroll
                        for (int jb = 0; jb < J; ++jb) {
                            acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xh[jb], acc[t][jb], 0, 0, 0);
                            acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xm[jb], acc[t][jb], 0, 0, 0);
                            acc[t][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, xl[jb], acc[t][jb], 0, 0, 0);
                        }
                    }
                }
            }
        }
    }

    if constexpr (NT > 0) {
        // ragged tail rows rows_main .. p-1 (fewer than one slot), FP32 FMA
        if (rows_main < p) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int64_t col = c0 + 16 * t + 4 * lk + v;
                    col = (col < cend) ? col : cend - 1;
                    const uint8_t* ac = Ab + col * colbytes;
                    for (int r = rows_main; r < p; ++r) {
                        const float a = (ST == kStBF16)
                                            ? bf16_value(reinterpret_cast<const uint16_t*>(ac)[r])
                                            : e4m3_value(ac[r]);
#pragma unroll
                        for (int jb = 0; jb < J; ++jb)
                            acc[t][jb][v] = __builtin_fmaf(a, xcol[jb][r], acc[t][jb][v]);
                    }
                }
        }
        // scale, threshold, S, activity flags
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t col = c0 + 16 * t + 4 * lk + v;
                const bool cvalid = col < cend;
                const float sc = cvalid ? column_scale(pp, col) : 1.0f;
                bool any = false;
#pragma unroll
                for (int jb = 0; jb < J; ++jb) {
                    const int comp = 16 * jb + lj;
                    if (cvalid && comp < m) {
                        float s;
                        double fv;
                        const bool a = thresh_q(l0, pp.mu[comp], pp.gam[comp], sc * acc[t][jb][v],
                                                s, fv);
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

template <int ST, int J, int STAGES, int TMAX>
__global__ __launch_bounds__(256) void k_corr_qw(PassParams pp, const float* __restrict__ X,
                                                 const float* __restrict__ Xil,
                                                 float* __restrict__ S, uint8_t* __restrict__ act,
                                                 double* __restrict__ fpart,
                                                 int* __restrict__ nnzpart,
                                                 const Ctrl* __restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int EPS = (ST == kStBF16) ? 8 : 16;
    constexpr int XBlk = 2 * EPS * 16 * 16;
    constexpr int StageBytes = 4 * TMAX * 2048 + J * XBlk;
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
#define GPSPCA_QW(NT) qw_round<NT, ST, J, STAGES, TMAX>(pp, c0, cend, lbase, wv, xcol, Xil, f_acc, nnz_acc, S, act)
        switch (k) {
            case 0: GPSPCA_QW(0); break;
            case 1: GPSPCA_QW(1); break;
            case 2: GPSPCA_QW(2); break;
            case 3: GPSPCA_QW(3); break;
            case 4: GPSPCA_QW(4); break;
            case 5: if constexpr (TMAX >= 5) GPSPCA_QW(5); break;
            case 6: if constexpr (TMAX >= 6) GPSPCA_QW(6); break;
            case 7: if constexpr (TMAX >= 7) GPSPCA_QW(7); break;
            default: if constexpr (TMAX >= 8) GPSPCA_QW(8); break;
        }
#undef GPSPCA_QW
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

// ------------------------------------------------------------- launchers
hipError_t launch_quantize(const float* A, int64_t lda, int p, int64_t n, int to, void* out,
                           int64_t ldq, float* scale, hipStream_t st) {
    const dim3 grid((unsigned)((n + 3) / 4)), block(256);
    if (to == GPSPCA_BF16)
        hipLaunchKernelGGL(k_quantize<kStBF16>, grid, block, 0, st, A, lda, p, n, out, ldq, scale);
    else
        hipLaunchKernelGGL(k_quantize<kStF8>, grid, block, 0, st, A, lda, p, n, out, ldq, scale);
    return hipGetLastError();
}

// Component blocks of the quantized kernel, and the stage counts it is built
// for: (storage, J) -> {2, 3, 8} for bfloat16 with J <= 2, {2, 8} for e4m3
// with J <= 2, else {2}.
static int q_blocks(int m) { return m <= 16 ? 1 : m <= 32 ? 2 : 4; }

// "8": 2 stages of chunks of up to 8 tiles, half the X instructions per byte
// of A -- the bfloat16 default for J <= 2 (24% faster at J = 2); e4m3 keeps
// 4-tile chunks (its 8-tile stages leave room for only two waves per CU, 10%
// slower at J = 2).
int corr_q_stages(int dtype, int m, int want) {
    const int J = q_blocks(m);
    if (dtype == GPSPCA_BF16 && J <= 2) return (want == 2 || want == 3) ? want : 8;
    if (J <= 2 && want == 8) return 8;
    return 2;
}

template <int ST, int J, int S, int TMAX = 4>
static int occ_q() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_corr_q<ST, J, S, TMAX>, 64, 0) !=
        hipSuccess)
        nb = 1;
    (void)hipGetLastError();
    return nb;
}

static int corr_q_blocks_per_cu_query(int dtype, int m, int stages);

// Cached per (storage, component groups, stages), as corr_mfma_blocks_per_cu.
int corr_q_blocks_per_cu(int dtype, int m, int stages) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int>, int> cache;
    const std::tuple<int, int, int> key(dtype, q_blocks(m), stages);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int nb = corr_q_blocks_per_cu_query(dtype, m, stages);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = nb;
    return nb;
}

static int corr_q_blocks_per_cu_query(int dtype, int m, int stages) {
    const int J = q_blocks(m);
    int nb;
    if (stages == 8 && J <= 2) {
        if (dtype == GPSPCA_BF16) nb = J == 1 ? occ_q<kStBF16, 1, 2, 8>() : occ_q<kStBF16, 2, 2, 8>();
        else nb = J == 1 ? occ_q<kStF8, 1, 2, 8>() : occ_q<kStF8, 2, 2, 8>();
    } else if (dtype == GPSPCA_BF16) {
        if (J == 1) nb = stages == 2 ? occ_q<kStBF16, 1, 2>() : occ_q<kStBF16, 1, 3>();
        else if (J == 2) nb = stages == 2 ? occ_q<kStBF16, 2, 2>() : occ_q<kStBF16, 2, 3>();
        else nb = occ_q<kStBF16, 4, 2>();
    } else {
        if (J == 1) nb = occ_q<kStF8, 1, 2>();
        else if (J == 2) nb = occ_q<kStF8, 2, 2>();
        else nb = occ_q<kStF8, 4, 2>();
    }
    return std::max(1, nb);
}

hipError_t launch_corr_q(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                         float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                         hipStream_t st) {
    const int J = q_blocks(pl.m), Sg = pl.mfma_stages;
    const dim3 grid(pl.corr_grid), block(64);
#define GPSPCA_CQ(STT, JJ, SS) \
    GPSPCA_LAUNCH_TIMED((k_corr_q<STT, JJ, SS>), grid, block, 0, st, pp, X, Xil, S, act, fpart, \
                       nnzpart, ctrl)
#define GPSPCA_CQW(STT, JJ) \
    GPSPCA_LAUNCH_TIMED((k_corr_q<STT, JJ, 2, 8>), grid, block, 0, st, pp, X, Xil, S, act, fpart, \
                       nnzpart, ctrl)
    if (Sg == 8 && J <= 2) {
        if (pl.dtype == GPSPCA_BF16) {
            if (J == 1) GPSPCA_CQW(kStBF16, 1);
            else GPSPCA_CQW(kStBF16, 2);
        } else {
            if (J == 1) GPSPCA_CQW(kStF8, 1);
            else GPSPCA_CQW(kStF8, 2);
        }
    } else if (pl.dtype == GPSPCA_BF16) {
        if (J == 1 && Sg == 2) GPSPCA_CQ(kStBF16, 1, 2);
        else if (J == 1) GPSPCA_CQ(kStBF16, 1, 3);
        else if (J == 2 && Sg == 2) GPSPCA_CQ(kStBF16, 2, 2);
        else if (J == 2) GPSPCA_CQ(kStBF16, 2, 3);
        else GPSPCA_CQ(kStBF16, 4, 2);
    } else {
        if (J == 1) GPSPCA_CQ(kStF8, 1, 2);
        else if (J == 2) GPSPCA_CQ(kStF8, 2, 2);
        else GPSPCA_CQ(kStF8, 4, 2);
    }
#undef GPSPCA_CQW
#undef GPSPCA_CQ
    return hipGetLastError();
}

// Four-wave workgroups sharing X (one per CU: their stages take 96-160 KB of
// LDS).  Shapes (chunk tiles per wave, stages): (8, 2) by default for J <= 2,
// (4, 3) for pl.mfma_stages = 3, (4, 2) for e4m3 with pl.mfma_stages = 2,
// and (4, 2) for J = 4.  On the 32-gamma path at 10000 x 100000: bfloat16
// 433 us with (8, 2) against 508 with (4, 3); e4m3 349 / 407 / 417 us with
// (8, 2) / (4, 2) / (4, 3); one wave per workgroup (k_corr_q) 529 and 516 us.
hipError_t launch_corr_qw(const Plan& pl, const PassParams& pp, const float* X, const float* Xil,
                          float* S, uint8_t* act, double* fpart, int* nnzpart, const Ctrl* ctrl,
                          hipStream_t st) {
    const int J = q_blocks(pl.m), Sg = pl.mfma_stages;
    const dim3 grid(pl.corr_grid), block(256);
#define GPSPCA_QWL(STT, JJ, SS, TT) \
    GPSPCA_LAUNCH_TIMED((k_corr_qw<STT, JJ, SS, TT>), grid, block, 0, st, pp, X, Xil, S, act, \
                       fpart, nnzpart, ctrl)
    if (pl.dtype == GPSPCA_BF16) {
        if (J == 1) {
            if (Sg == 3) GPSPCA_QWL(kStBF16, 1, 3, 4); else GPSPCA_QWL(kStBF16, 1, 2, 8);
        } else if (J == 2) {
            if (Sg == 3) GPSPCA_QWL(kStBF16, 2, 3, 4); else GPSPCA_QWL(kStBF16, 2, 2, 8);
        } else {
            GPSPCA_QWL(kStBF16, 4, 2, 4);
        }
    } else {
        if (J == 1) {
            if (Sg == 3) GPSPCA_QWL(kStF8, 1, 3, 4);
            else if (Sg == 2) GPSPCA_QWL(kStF8, 1, 2, 4);
            else GPSPCA_QWL(kStF8, 1, 2, 8);
        } else if (J == 2) {
            if (Sg == 3) GPSPCA_QWL(kStF8, 2, 3, 4);
            else if (Sg == 2) GPSPCA_QWL(kStF8, 2, 2, 4);
            else GPSPCA_QWL(kStF8, 2, 2, 8);
        } else {
            GPSPCA_QWL(kStF8, 4, 2, 4);
        }
    }
#undef GPSPCA_QWL
    return hipGetLastError();
}

}  // namespace gpspca
