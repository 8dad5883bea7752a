// Split-BF16 GEMM tile engine shared by the one-problem kernel, the split-K
// path and the persistent batched kernel (Sec. II-D, II-G, IV-A).
//
// One call computes a BM x BN tile of C = alpha A B + beta C over the K range
// [kb, ke).  Per K-step of 32:
//   1. FP32 tiles of A (BM x 32) and B (32 x BN) are loaded from global memory
//      with 16-byte coalesced loads one step ahead and held in registers;
//   2. every value is split into P = 1, 2 or 3 BF16 terms in registers
//      (Sec. II-A) and the planes are stored to LDS k-contiguous for both
//      operands (B is transposed on the way), double-buffered;
//   3. v_mfma_f32_16x16x32_bf16 runs over the plane pairs of the variant: the
//      products of bins 4..1 accumulate into an FP32 "lo" accumulator,
//      smallest bin first, A0 x B0 (bin 0) into a "hi" accumulator.
// The epilogue forms X = hi + lo (the largest bin added last, Sec. II-G) and
// writes C = alpha X (beta == 0: C not read) or fma(alpha, X, beta C), or, for
// split-K, the hi and lo partial sums.
#pragma once

#include "common.hpp"

namespace bfx {

// (i, j) plane pairs of the lo accumulator, in issue order (bins 4 -> 1).
// Bin 0 (0,0) always goes to hi.
template <int V> struct Prods;
template <> struct Prods<1> {
    static constexpr int P = 1, n = 0;
    static constexpr int ai[1] = {0}, bj[1] = {0};
};
template <> struct Prods<3> {
    static constexpr int P = 2, n = 2;
    static constexpr int ai[2] = {1, 0}, bj[2] = {0, 1};
};
template <> struct Prods<6> {
    static constexpr int P = 3, n = 5;
    static constexpr int ai[5] = {2, 1, 0, 1, 0}, bj[5] = {0, 1, 2, 0, 1};
};
template <> struct Prods<9> {
    static constexpr int P = 3, n = 8;
    static constexpr int ai[8] = {2, 2, 1, 2, 1, 0, 1, 0};
    static constexpr int bj[8] = {2, 1, 2, 0, 1, 2, 0, 1};
};

struct GemmParams {
    int64_t M, N, K;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    float alpha, beta;
    int64_t k_per_split;  // multiple of 32; K range of one split
    int splits;           // 1 = direct epilogue
    float *partial;       // [splits][2][M][N] when splits > 1
    int vecA, vecB;       // 16-byte loads allowed
};

constexpr int BK = 32;
constexpr int LDK = BK + 8;  // LDS row length in BF16 (80 bytes: conflict-free 16 B reads)

// Bijective remap of the launch index so that the workgroups resident on one
// XCD (hardware places workgroup i on XCD i % 8) get consecutive tile ids.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t total) {
    const int64_t q = total / 8, r = total % 8;
    const int64_t xcd = bid % 8, slot = bid / 8;
    return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// LDS bytes one tile call needs.
template <int V, int BM, int BN>
constexpr size_t tile_lds_bytes() {
    return 2ull * Prods<V>::P * (BM + BN) * LDK * sizeof(uint16_t);
}

// Computes one BM x BN output tile at (m0, n0) over K range [kb, ke).
// All WM*WN*64 threads of the workgroup must call it (it synchronises).
// split >= 0 with p.splits > 1 writes hi/lo partials of that split.
template <int V, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void gemm_tile(const GemmParams &p, int64_t m0, int64_t n0,
                                          int64_t kb, int64_t ke, int64_t split,
                                          uint16_t *smem) {
    using PR = Prods<V>;
    constexpr int P = PR::P;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM / 16;
    constexpr int TN = BN / WN / 16;
    constexpr int A_TOT = BM * BK / 4;              // float4 pieces of the A tile
    constexpr int B_TOT = (BK / 4) * (BN / 4);      // 4(k) x 4(n) blocks of the B tile
    constexpr int A_F4 = (A_TOT + NT - 1) / NT;     // per thread (guarded)
    constexpr int B_BLK = (B_TOT + NT - 1) / NT;
    constexpr int PLANE = (BM + BN) * LDK;        // BF16 elements per plane

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    const int64_t KT = (ke > kb) ? ceil_div(ke - kb, BK) : 0;

    float ra[A_F4][4];
    float rb[B_BLK][4][4];

    auto load_tile = [&](int64_t k0) {
#pragma unroll
        for (int i = 0; i < A_F4; ++i) {
            const int f = tid + i * NT;
            if (A_TOT % NT != 0 && f >= A_TOT) break;
            const int row = f / (BK / 4), kq = f % (BK / 4);
            const int64_t gm = m0 + row, gk = k0 + kq * 4;
            const float *src = p.A + gm * p.lda + gk;
            if (gm < p.M && gk + 4 <= ke && p.vecA) {
                const float4 v = *reinterpret_cast<const float4 *>(src);
                ra[i][0] = v.x; ra[i][1] = v.y; ra[i][2] = v.z; ra[i][3] = v.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    ra[i][j] = (gm < p.M && gk + j < ke) ? src[j] : 0.0f;
            }
        }
#pragma unroll
        for (int i = 0; i < B_BLK; ++i) {
            const int f = tid + i * NT;
            if (B_TOT % NT != 0 && f >= B_TOT) break;
            const int n4 = f % (BN / 4), k4 = f / (BN / 4);
            const int64_t gn = n0 + n4 * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t gk = k0 + k4 * 4 + j;
                const float *src = p.B + gk * p.ldb + gn;
                if (gk < ke && gn + 4 <= p.N && p.vecB) {
                    const float4 v = *reinterpret_cast<const float4 *>(src);
                    rb[i][j][0] = v.x; rb[i][j][1] = v.y; rb[i][j][2] = v.z; rb[i][j][3] = v.w;
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        rb[i][j][c] = (gk < ke && gn + c < p.N) ? src[c] : 0.0f;
                }
            }
        }
    };

    auto store_tile = [&](int buf) {
        uint16_t *base = smem + buf * P * PLANE;
#pragma unroll
        for (int i = 0; i < A_F4; ++i) {
            const int f = tid + i * NT;
            if (A_TOT % NT != 0 && f >= A_TOT) break;
            const int row = f / (BK / 4), kq = f % (BK / 4);
            uint32_t h[3][2];
            split4<P>(ra[i], h);
#pragma unroll
            for (int pl = 0; pl < P; ++pl)
                *reinterpret_cast<uint2 *>(base + pl * PLANE + row * LDK + kq * 4) =
                    make_uint2(h[pl][0], h[pl][1]);
        }
#pragma unroll
        for (int i = 0; i < B_BLK; ++i) {
            const int f = tid + i * NT;
            if (B_TOT % NT != 0 && f >= B_TOT) break;
            const int n4 = f % (BN / 4), k4 = f / (BN / 4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const float col[4] = {rb[i][0][c], rb[i][1][c], rb[i][2][c], rb[i][3][c]};
                uint32_t h[3][2];
                split4<P>(col, h);
                const int n = n4 * 4 + c;
#pragma unroll
                for (int pl = 0; pl < P; ++pl)
                    *reinterpret_cast<uint2 *>(base + pl * PLANE + (BM + n) * LDK + k4 * 4) =
                        make_uint2(h[pl][0], h[pl][1]);
            }
        }
    };

    bfx_f32x4 hi[TM][TN], lo[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            hi[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
            lo[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
        }

    const int r16 = lane & 15, kg = lane >> 4;
    auto compute = [&](int buf) {
        const uint16_t *base = smem + buf * P * PLANE;
        bfx_bf16x8 af[P][TM], bf[P][TN];
#pragma unroll
        for (int pl = 0; pl < P; ++pl) {
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm * TM * 16 + i * 16 + r16;
                af[pl][i] = *reinterpret_cast<const bfx_bf16x8 *>(base + pl * PLANE + row * LDK + kg * 8);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int n = wn * TN * 16 + j * 16 + r16;
                bf[pl][j] = *reinterpret_cast<const bfx_bf16x8 *>(base + pl * PLANE + (BM + n) * LDK + kg * 8);
            }
        }
#pragma unroll
        for (int q = 0; q < PR::n; ++q)
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        af[PR::ai[q]][i], bf[PR::bj[q]][j], lo[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                hi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[0][j],
                                                                    hi[i][j], 0, 0, 0);
    };

    if (KT > 0) {
        load_tile(kb);
        store_tile(0);
        __syncthreads();
        for (int64_t s = 0; s < KT; ++s) {
            const int cur = (int)(s & 1);
            if (s + 1 < KT) load_tile(kb + (s + 1) * BK);
            compute(cur);
            if (s + 1 < KT) store_tile(cur ^ 1);
            __syncthreads();
        }
    }

    // Output layout of v_mfma_f32_16x16x32_bf16: lane holds column lane%16,
    // rows 4*(lane/16) + 0..3 of the 16x16 tile.
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + wm * TM * 16 + i * 16 + kg * 4 + e;
                const int64_t col = n0 + wn * TN * 16 + j * 16 + r16;
                if (row >= p.M || col >= p.N) continue;
                if (p.splits > 1) {
                    float *dst = p.partial + (split * 2) * p.M * p.N + row * p.N + col;
                    dst[0] = hi[i][j][e];
                    dst[p.M * p.N] = lo[i][j][e];
                } else {
                    const float X = hi[i][j][e] + lo[i][j][e];
                    float *c = p.C + row * p.ldc + col;
                    *c = (p.beta == 0.0f) ? p.alpha * X : fmaf(p.alpha, X, p.beta * *c);
                }
            }
}


}  // namespace bfx
