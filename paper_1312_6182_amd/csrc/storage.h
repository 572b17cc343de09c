// Device helpers for the storage types of A: FP32, bfloat16 and OCP float8
// e4m3fn with per-column FP32 scales.  A quantized column holds codes q_ri;
// its values are scale_i * value(q_ri), and every kernel applies scale_i to
// the column's dot products and back-projection weights rather than to each
// element.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpspca_internal.h"

namespace gpspca {

enum { kStF32 = 0, kStBF16 = 1, kStF8 = 2 };

typedef float qf4 __attribute__((ext_vector_type(4)));
typedef float qf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf16_value(uint32_t code16) {
    return __uint_as_float(code16 << 16);
}

// Two e4m3fn codes (bytes 0,1 or 2,3 of w) to FP32, by the gfx950 converter.
__device__ __forceinline__ qf2 e4m3_pair(uint32_t w, bool high) {
    return high ? __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true)
                : __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
}

__device__ __forceinline__ float e4m3_value(uint32_t code8) {
    return __builtin_amdgcn_cvt_f32_fp8((int)code8, 0);
}

// Base address of column `col` in bytes-typed storage.
template <int ST>
__device__ __forceinline__ const void* column_ptr(const PassParams& pp, int64_t col) {
    if constexpr (ST == kStBF16) return pp.Abf + col * pp.lda;
    else if constexpr (ST == kStF8) return pp.Af8 + col * pp.lda;
    else return pp.A + col * pp.lda;
}

// Unscaled values of rows 4q .. 4q+3 of a column; rows >= p read as 0.  Full
// quads use one 16-, 8- or 4-byte load (lda is a multiple of 4 and the base is
// aligned on every path that calls this with q < nqf).
template <int ST>
__device__ __forceinline__ qf4 load_quad_st(const void* colv, int q, int nqf, int p) {
    const int r = 4 * q;
    if constexpr (ST == kStF32) {
        const float* col = static_cast<const float*>(colv);
        if (q < nqf) return __builtin_nontemporal_load(reinterpret_cast<const qf4*>(col + r));
        qf4 v = qf4{0.f, 0.f, 0.f, 0.f};
        if (r < p) v.x = col[r];
        if (r + 1 < p) v.y = col[r + 1];
        if (r + 2 < p) v.z = col[r + 2];
        if (r + 3 < p) v.w = col[r + 3];
        return v;
    } else if constexpr (ST == kStBF16) {
        const uint16_t* col = static_cast<const uint16_t*>(colv);
        if (q < nqf) {
            const uint2 w = *reinterpret_cast<const uint2*>(col + r);
            return qf4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                       __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u)};
        }
        qf4 v = qf4{0.f, 0.f, 0.f, 0.f};
        if (r < p) v.x = bf16_value(col[r]);
        if (r + 1 < p) v.y = bf16_value(col[r + 1]);
        if (r + 2 < p) v.z = bf16_value(col[r + 2]);
        if (r + 3 < p) v.w = bf16_value(col[r + 3]);
        return v;
    } else {
        const uint8_t* col = static_cast<const uint8_t*>(colv);
        if (q < nqf) {
            const uint32_t w = *reinterpret_cast<const uint32_t*>(col + r);
            const qf2 lo = e4m3_pair(w, false), hi = e4m3_pair(w, true);
            return qf4{lo.x, lo.y, hi.x, hi.y};
        }
        qf4 v = qf4{0.f, 0.f, 0.f, 0.f};
        if (r < p) v.x = e4m3_value(col[r]);
        if (r + 1 < p) v.y = e4m3_value(col[r + 1]);
        if (r + 2 < p) v.z = e4m3_value(col[r + 2]);
        if (r + 3 < p) v.w = e4m3_value(col[r + 3]);
        return v;
    }
}

// Adds the active-column counts c held by the lanes of this wave to *nact (one
// integer atomic per wave, so the total does not depend on the order).  Called
// by every lane of the wave.
__device__ __forceinline__ void add_active_count(int c, int* nact) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c > 0 && nact) atomicAdd(nact, c);
}

// Scale of column `col` (1 when the matrix has none).
__device__ __forceinline__ float column_scale(const PassParams& pp, int64_t col) {
    return pp.scale ? pp.scale[col] : 1.0f;
}

}  // namespace gpspca
