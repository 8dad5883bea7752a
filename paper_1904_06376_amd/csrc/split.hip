// Standalone split (Sec. II-A): FP32 array -> two or three BF16 planes.
// Memory-bound: 4 bytes read and 4 or 6 bytes written per element.  Each
// thread converts four consecutive values with one 16-byte load and one
// 8-byte store per plane; the bit-exact integer conversion is used for every
// element (the arithmetic is far below the HBM time).
#include "common.hpp"

namespace bfx {

template <int P>
__global__ void __launch_bounds__(256)
split_kernel(const float *__restrict__ a, int64_t n, uint16_t *__restrict__ b0,
             uint16_t *__restrict__ b1, uint16_t *__restrict__ b2, bool vec) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n;
         i += stride) {
        uint16_t *out[3] = {b0, b1, b2};
        if (vec && i + 4 <= n) {
            const float4 v = *reinterpret_cast<const float4 *>(a + i);
            const float e[4] = {v.x, v.y, v.z, v.w};
            uint32_t h[4][3];
#pragma unroll
            for (int j = 0; j < 4; ++j) split3_exact(e[j], h[j][0], h[j][1], h[j][2]);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                uint2 w;
                w.x = h[0][p] | (h[1][p] << 16);
                w.y = h[2][p] | (h[3][p] << 16);
                *reinterpret_cast<uint2 *>(out[p] + i) = w;
            }
        } else {
            const int64_t e = (i + 4 <= n) ? i + 4 : n;
            for (int64_t j = i; j < e; ++j) {
                uint32_t h[3];
                split3_exact(a[j], h[0], h[1], h[2]);
#pragma unroll
                for (int p = 0; p < P; ++p) out[p][j] = (uint16_t)h[p];
            }
        }
    }
}

}  // namespace bfx

extern "C" int bfx_split_f32(const float *a, int64_t n, int nterms, uint16_t *b0,
                             uint16_t *b1, uint16_t *b2, void *stream) {
    if (n < 0) return -2;
    if (nterms != 2 && nterms != 3) return -3;
    if (n == 0) return BFX_OK;
    if (!a) return -1;
    if (!b0) return -4;
    if (!b1) return -5;
    if (nterms == 3 && !b2) return -6;
    const bool vec = ((uintptr_t)a % 16 == 0) && ((uintptr_t)b0 % 8 == 0) &&
                     ((uintptr_t)b1 % 8 == 0) &&
                     (nterms == 2 || (uintptr_t)b2 % 8 == 0);
    const int64_t quads = bfx::ceil_div(n, 4);
    int64_t blocks = bfx::ceil_div(quads, 256);
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipStream_t s = (hipStream_t)stream;
    if (nterms == 3)
        hipLaunchKernelGGL(bfx::split_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s,
                           a, n, b0, b1, b2, vec);
    else
        hipLaunchKernelGGL(bfx::split_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s,
                           a, n, b0, b1, b2, vec);
    BFX_LAUNCH_CHECK("split_kernel launch");
    return BFX_OK;
}
