// Device and host helpers shared by the libbfx kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "bfx.h"

typedef __bf16 bfx_bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bfx_bf16x2 __attribute__((ext_vector_type(2)));
typedef float bfx_f32x2 __attribute__((ext_vector_type(2)));
typedef float bfx_f32x4 __attribute__((ext_vector_type(4)));
typedef float bfx_f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t bfx_u32x4 __attribute__((ext_vector_type(4)));

namespace bfx {

// ---------------------------------------------------------------------------
// FP32 -> BF16 conversion (Sec. I, II-A) with the library's rules:
// round to nearest even on the bit pattern, saturate finite overflow to the
// largest BF16 of that sign, canonical quiet NaN, subnormals kept.
// Result: the 16-bit pattern in the low half of the return value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bf16_bits_exact(float a) {
    const uint32_t u = __float_as_uint(a);
    const uint32_t mag = u & 0x7fffffffu;
    const uint32_t sgn16 = (u >> 16) & 0x8000u;
    uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    if (mag >= 0x7f800000u)
        r = (mag == 0x7f800000u) ? (u >> 16) : (sgn16 | 0x7fc0u);
    else if ((r & 0x7fffu) == 0x7f80u)
        r = sgn16 | 0x7f7fu;
    return r;
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) {
    return __uint_as_float(h << 16);
}

// Sec. II-A split, exact for every input (including subnormal, overflow
// and non-finite cases): b0 = (B16)a, b1 = (B16)(a-b0), b2 = (B16)(a-b0-b1).
__device__ __forceinline__ void split3_exact(float a, uint32_t &h0,
                                             uint32_t &h1, uint32_t &h2) {
    h0 = bf16_bits_exact(a);
    if ((__float_as_uint(a) & 0x7fffffffu) >= 0x7f800000u) {
        h1 = 0u;
        h2 = 0u;
        return;
    }
    const float r1 = a - bf16_bits_to_f32(h0);
    h1 = bf16_bits_exact(r1);
    const float r2 = r1 - bf16_bits_to_f32(h1);
    h2 = bf16_bits_exact(r2);
}

// Hardware round-to-nearest-even conversion of two FP32 values into one
// packed BF16 pair (low half = lo).  Equal to bf16_bits_exact for zeros and
// finite normal values below the saturation threshold.
__device__ __forceinline__ uint32_t cvt_pk_bf16(float lo, float hi) {
    bfx_f32x2 v = {lo, hi};
    bfx_bf16x2 r = __builtin_convertvector(v, bfx_bf16x2);
    return __builtin_bit_cast(uint32_t, r);
}

// A value is "tame" when it is zero or 2^-100 <= |a| < 0x7F7F8000: then
// every intermediate of its split is zero or a normal FP32 number and no
// term saturates, so the hardware conversion gives the exact split.
__device__ __forceinline__ bool split_tame(float a) {
    const uint32_t mag = __float_as_uint(a) & 0x7fffffffu;
    return mag == 0u || (mag - 0x0d800000u) < (0x7f7f8000u - 0x0d800000u);
}

// Split of a pair of tame values into packed BF16 planes (low half = x).
template <int P>
__device__ __forceinline__ void split_pair_fast(float x, float y, uint32_t *p) {
    p[0] = cvt_pk_bf16(x, y);
    if constexpr (P > 1) {
        const float rx = x - __uint_as_float(p[0] << 16);
        const float ry = y - __uint_as_float(p[0] & 0xffff0000u);
        p[1] = cvt_pk_bf16(rx, ry);
        if constexpr (P > 2) {
            const float sx = rx - __uint_as_float(p[1] << 16);
            const float sy = ry - __uint_as_float(p[1] & 0xffff0000u);
            p[2] = cvt_pk_bf16(sx, sy);
        }
    }
}

template <int P>
__device__ __forceinline__ void split_pair_exact(float x, float y, uint32_t *p) {
    uint32_t hx[3], hy[3];
    split3_exact(x, hx[0], hx[1], hx[2]);
    split3_exact(y, hy[0], hy[1], hy[2]);
#pragma unroll
    for (int i = 0; i < P; ++i) p[i] = hx[i] | (hy[i] << 16);
}

// Split four consecutive values into P planes of packed pairs:
// out[plane][0] = (v0,v1), out[plane][1] = (v2,v3).  The fast path is taken
// when all four are tame; otherwise the exact integer path.
template <int P>
__device__ __forceinline__ void split4(const float v[4], uint32_t out[][2]) {
    const bool tame = (int)split_tame(v[0]) & (int)split_tame(v[1]) & (int)split_tame(v[2]) &
                      (int)split_tame(v[3]);
    uint32_t a[3], b[3];
    if (__builtin_expect(tame, 1)) {
        split_pair_fast<P>(v[0], v[1], a);
        split_pair_fast<P>(v[2], v[3], b);
    } else {
        split_pair_exact<P>(v[0], v[1], a);
        split_pair_exact<P>(v[2], v[3], b);
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        out[i][0] = a[i];
        out[i][1] = b[i];
    }
}

// ---------------------------------------------------------------------------
// Host-side error plumbing.
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define BFX_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return bfx::hip_fail(e_, #call); \
    } while (0)

#define BFX_LAUNCH_CHECK(what)                         \
    do {                                               \
        hipError_t e_ = hipGetLastError();             \
        if (e_ != hipSuccess) return bfx::hip_fail(e_, what); \
    } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Internal GEMM launcher shared by the public entry points, the LU trailing
// update and the batched per-problem baseline.  grid_cus > 0: the stream's
// kernels run on that many compute units (a CU-masked stream), which sizes
// the persistent launch; 0: the whole device.
int gemm_launch(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                const float *A, int64_t lda, const float *B, int64_t ldb,
                float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                hipStream_t stream, int flags = 0, int grid_cus = 0);
// 1, 3, 6, 7, 8, 9 and the per-operand split counts 12, 13, 21, 23, 31, 32.
bool variant_valid(int variant);
size_t gemm_ws_bytes(int variant, int64_t M, int64_t N, int64_t K);

}  // namespace bfx
