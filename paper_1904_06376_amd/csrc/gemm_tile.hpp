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


// ---------------------------------------------------------------------------
// Fast path: BM x BN tile (128 x 128 or 64 x 64), 4 MFMA + 4 helper waves.
// Requirements: A rows 16-byte aligned (A 16-byte aligned, lda % 4 == 0),
// K % 4 == 0 and the K range of a split a multiple of 32.  M, N and K need
// not fill the tile: partial tiles are handled by clamped loads whose values
// are replaced by zeros and by a masked epilogue.  Differences from gemm_tile:
//   * loads: one thread per A row / B column and BM*32/256 consecutive k
//     values (16-byte loads of A, coalesced 4-byte loads of B) through buffer
//     resources, so every LDS store is a conflict-free 16-byte store of 8 BF16
//     (rows are 80 bytes apart);
//   * global loads are issued two K-steps ahead (two register stages);
//   * the split is branch-free (hardware RNE); the rare values for which it is
//     not exact (Inf/NaN, or a first term that rounds to Inf) are detected from
//     the first plane and re-split exactly afterwards, outside the MFMA block,
//     from a second read of global memory, so loads, split and MFMA of one
//     K-step form a single basic block.
// ---------------------------------------------------------------------------

// Packed BF16 pairs of KPT consecutive values -> P planes x KPT/2 dwords.
// `flag` collects (per 16-bit half, unsigned max) the magnitude of every
// first term: a half >= 0x7F80 marks an Inf/NaN first term.
template <int P, int KPT>
__device__ __forceinline__ void split_run_fast(const float *v, uint32_t out[][KPT / 2], uint32_t &flag) {
#pragma unroll
    for (int i = 0; i < KPT / 2; ++i) {
        uint32_t t[3];
        split_pair_fast<P>(v[2 * i], v[2 * i + 1], t);
#pragma unroll
        for (int pl = 0; pl < P; ++pl) out[pl][i] = t[pl];
        typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
        const u16x2 m = __builtin_bit_cast(u16x2, t[0] & 0x7fff7fffu);
        flag = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, flag), m));
    }
}

__device__ __forceinline__ bool flag_bad(uint32_t flag) {
    return (flag & 0xffffu) >= 0x7f80u || (flag >> 16) >= 0x7f80u;
}

// Wave-specialised aligned tile: 512 threads.  Waves 0-3 (one per SIMD) only
// read BF16 fragments from LDS, run the MFMAs and write the epilogue; waves
// 4-7 (one per SIMD) only load FP32 tiles (two K-steps ahead), split them and
// store the planes.  Every SIMD thus runs one wave of each kind and overlaps
// the split's VALU work with the other wave's matrix work.  Both kinds pass
// the same barrier once per K-step; the LDS planes are double-buffered.
template <int V, int BM, int BN>
__device__ __forceinline__ void gemm_tile_fast(const GemmParams &p, int64_t m0, int64_t n0,
                                               int64_t kb, int64_t ke, int64_t split,
                                               uint16_t *smem) {
    using PR = Prods<V>;
    constexpr int P = PR::P;
    constexpr int PLANE = (BM + BN) * LDK;
    constexpr int TM = BM / 32, TN = BN / 32;          // 16x16 tiles per MFMA wave (2 x 2 waves)
    constexpr int KPT = BM * BK / 256;                  // k values per helper thread
    static_assert(BM == BN && KPT % 8 == 0, "square tiles with >= 8 k values per helper thread");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int KT = (int)ceil_div(ke - kb, (int64_t)BK);

    if (wave < 4) {
        // ------------------------------ MFMA waves ------------------------------
        const int wm = wave >> 1, wn = wave & 1;
        bfx_f32x4 hi[TM][TN], lo[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                hi[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
                lo[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
            }
        const int r16 = lane & 15, kg = lane >> 4;
        for (int s = 0; s < KT; ++s) {
            __syncthreads();  // buffer s&1 holds step s
            const uint16_t *base = smem + (s & 1) * P * PLANE;
            bfx_bf16x8 af[P][TM];
#pragma unroll
            for (int pl = 0; pl < P; ++pl)
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    af[pl][i] = *reinterpret_cast<const bfx_bf16x8 *>(
                        base + pl * PLANE + (wm * (BM / 2) + i * 16 + r16) * LDK + kg * 8);
            // B fragments one plane at a time (plane 2, 1, 0): within each B
            // plane the lo products are issued smallest bin first.
#pragma unroll
            for (int jp = P - 1; jp >= 0; --jp) {
                bfx_bf16x8 bf[TN];
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    bf[j] = *reinterpret_cast<const bfx_bf16x8 *>(
                        base + jp * PLANE + (BM + wn * (BN / 2) + j * 16 + r16) * LDK + kg * 8);
#pragma unroll
                for (int q = 0; q < PR::n; ++q) {
                    if (PR::bj[q] != jp) continue;
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            lo[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[PR::ai[q]][i], bf[j],
                                                                                lo[i][j], 0, 0, 0);
                }
                if (jp == 0) {
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            hi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[j],
                                                                                hi[i][j], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // matches the helpers' final barrier
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = m0 + wm * (BM / 2) + i * 16 + kg * 4 + e;
                    const int64_t col = n0 + wn * (BN / 2) + j * 16 + r16;
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
        return;
    }

    // ------------------------------ helper waves ------------------------------
    const int h = tid - 256;
    const int arow = h % BM, aq = h / BM;   // A row, k group
    const int bcol = h % BN, bq = h / BN;   // B column, k group
    // Extent of this tile inside the matrices.  `full` (uniform) selects the
    // unmasked code; otherwise every load is clamped to an element inside the
    // tile's range and its value replaced by zero before the split.
    const int rows = (int)((p.M - m0 < BM) ? p.M - m0 : BM);
    const int cols = (int)((p.N - n0 < BN) ? p.N - n0 : BN);
    const int klen = (int)(ke - kb);
    const bool full = rows == BM && cols == BN && klen % BK == 0;
    const bool a_ok = arow < rows, b_ok = bcol < cols;
    // Buffer resources over exactly the elements of this tile's A rows and B
    // columns (the range check is a second guard; no load leaves the range).
    const int lda = (int)p.lda, ldb = (int)p.ldb;
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.A + m0 * p.lda + kb), (short)0, ((rows - 1) * lda + klen) * 4, 0x00020000);
    const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.B + kb * p.ldb + n0), (short)0, ((klen - 1) * ldb + cols) * 4, 0x00020000);
    const int voA = ((a_ok ? arow : 0) * lda + aq * KPT) * 4;
    const int voB = (bq * KPT * ldb + (b_ok ? bcol : 0)) * 4;

    float ra[2][KPT], rb[2][KPT];
    auto issue = [&](int st, int step) {
        if (full) {
            const int soA = step * BK * 4;
#pragma unroll
            for (int q = 0; q < KPT / 4; ++q) {
                const bfx_f32x4 v = __builtin_bit_cast(
                    bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, voA + 16 * q, soA, 0));
                ra[st][4 * q] = v[0]; ra[st][4 * q + 1] = v[1]; ra[st][4 * q + 2] = v[2]; ra[st][4 * q + 3] = v[3];
            }
            const int soB = step * BK * ldb * 4;
#pragma unroll
            for (int j = 0; j < KPT; ++j)
                rb[st][j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rB, voB, soB + j * ldb * 4, 0));
        } else {
            // k beyond the range: read k = 0 of the same row / column instead
            const int k0 = step * BK + aq * KPT;
#pragma unroll
            for (int q = 0; q < KPT / 4; ++q) {
                const int off = (k0 + 4 * q < klen) ? voA + (step * BK + 4 * q) * 4 : voA - aq * KPT * 4;
                const bfx_f32x4 v = __builtin_bit_cast(
                    bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, off, 0, 0));
                ra[st][4 * q] = v[0]; ra[st][4 * q + 1] = v[1]; ra[st][4 * q + 2] = v[2]; ra[st][4 * q + 3] = v[3];
            }
            const int kB = step * BK + bq * KPT;
#pragma unroll
            for (int j = 0; j < KPT; ++j) {
                const int off = (kB + j < klen) ? voB + (step * BK + j) * ldb * 4 : voB - bq * KPT * ldb * 4;
                rb[st][j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rB, off, 0, 0));
            }
        }
    };
    // Zeros for the values outside the tile (partial tiles only).
    auto mask = [&](int st, int step) {
        const int k0 = step * BK + aq * KPT, kB = step * BK + bq * KPT;
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            if (!a_ok || k0 + q >= klen) ra[st][q] = 0.0f;
            if (!b_ok || kB + q >= klen) rb[st][q] = 0.0f;
        }
    };
    auto put = [&](uint16_t *base, int row, int kg0, const uint32_t pl8[][KPT / 2]) {
#pragma unroll
        for (int pl = 0; pl < P; ++pl) {
            uint16_t *d = base + pl * PLANE + row * LDK + kg0 * KPT;
#pragma unroll
            for (int c = 0; c < KPT / 8; ++c)
                *reinterpret_cast<uint4 *>(d + 8 * c) =
                    make_uint4(pl8[pl][4 * c], pl8[pl][4 * c + 1], pl8[pl][4 * c + 2], pl8[pl][4 * c + 3]);
        }
    };
    auto stage = [&](int st, int buf, int step) {
        if (!full) mask(st, step);
        uint16_t *base = smem + buf * P * PLANE;
        uint32_t flag = 0, pa[3][KPT / 2], pb[3][KPT / 2];
        split_run_fast<P, KPT>(ra[st], pa, flag);
        split_run_fast<P, KPT>(rb[st], pb, flag);
        put(base, arow, aq, pa);
        put(base, BM + bcol, bq, pb);
        return flag;
    };
    // Rare path: re-read this thread's values of K-step `step` (still in L2)
    // and split them exactly, one BF16 store at a time.
    auto fixup = [&](int step, int buf) {
        uint16_t *base = smem + buf * P * PLANE;
#pragma unroll 1
        for (int e = 0; e < 2 * KPT; ++e) {
            const bool isA = e < KPT;
            const int q = isA ? e : e - KPT;
            const int k = (isA ? aq : bq) * KPT + q;
            const bool in = (isA ? a_ok : b_ok) && step * BK + k < klen;
            const uint32_t bits = !in ? 0u
                : isA ? __builtin_amdgcn_raw_buffer_load_b32(rA, voA + 4 * q, step * BK * 4, 0)
                      : __builtin_amdgcn_raw_buffer_load_b32(rB, voB, (step * BK + q) * ldb * 4, 0);
            uint32_t hh[3];
            split3_exact(__builtin_bit_cast(float, bits), hh[0], hh[1], hh[2]);
            const int row = isA ? arow : BM + bcol;
#pragma unroll
            for (int pl = 0; pl < P; ++pl) base[pl * PLANE + row * LDK + k] = (uint16_t)hh[pl];
        }
    };
    // Step t+1 is split into buffer (t+1)&1 while the MFMA waves work on step
    // t; its registers then receive the loads of step t+3.
#define BFX_HELPER_STEP(t, SP)                                             \
    {                                                                      \
        __syncthreads();                                                   \
        if ((t) + 1 < KT) {                                                \
            const uint32_t flag = stage(SP, ((t) + 1) & 1, (t) + 1);       \
            issue(SP, ((t) + 3 < KT) ? (t) + 3 : KT - 1);                  \
            if (flag_bad(flag)) fixup((t) + 1, ((t) + 1) & 1);             \
        }                                                                  \
    }
    if (KT > 0) {
        issue(0, 0);
        issue(1, KT > 1 ? 1 : KT - 1);
        const uint32_t flag = stage(0, 0, 0);
        issue(0, KT > 2 ? 2 : KT - 1);
        if (flag_bad(flag)) fixup(0, 0);
        int s = 0;
        for (; s + 1 < KT; s += 2) {
            BFX_HELPER_STEP(s, 1);
            BFX_HELPER_STEP(s + 1, 0);
        }
        if (s < KT) BFX_HELPER_STEP(s, 1);
    }
#undef BFX_HELPER_STEP
    __syncthreads();
}

}  // namespace bfx
