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

#include <type_traits>

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
// x7: x6 plus A1 B2 (bin 3); x8: all of bins 0-3 (Sec. II-D, IV-A).
template <> struct Prods<7> {
    static constexpr int P = 3, n = 6;
    static constexpr int ai[6] = {1, 2, 1, 0, 1, 0}, bj[6] = {2, 0, 1, 2, 0, 1};
};
template <> struct Prods<8> {
    static constexpr int P = 3, n = 7;
    static constexpr int ai[7] = {1, 2, 2, 1, 0, 1, 0}, bj[7] = {2, 1, 0, 1, 2, 0, 1};
};
template <> struct Prods<9> {
    static constexpr int P = 3, n = 8;
    static constexpr int ai[8] = {2, 2, 1, 2, 1, 0, 1, 0};
    static constexpr int bj[8] = {2, 1, 2, 0, 1, 2, 0, 1};
};
// Per-operand split counts (Sec. II-G): variant 10 pa + pb takes pa BF16
// terms of A and pb of B and the products a_i b_j, i < pa, j < pb,
// i + j <= 2.  P = max(pa, pb) planes of both operands are formed; the planes
// of the operand with fewer terms beyond its count are not used.
template <> struct Prods<12> {
    static constexpr int P = 2, n = 1;
    static constexpr int ai[1] = {0}, bj[1] = {1};
};
template <> struct Prods<21> {
    static constexpr int P = 2, n = 1;
    static constexpr int ai[1] = {1}, bj[1] = {0};
};
template <> struct Prods<13> {
    static constexpr int P = 3, n = 2;
    static constexpr int ai[2] = {0, 0}, bj[2] = {2, 1};
};
template <> struct Prods<31> {
    static constexpr int P = 3, n = 2;
    static constexpr int ai[2] = {2, 1}, bj[2] = {0, 0};
};
template <> struct Prods<23> {
    static constexpr int P = 3, n = 4;
    static constexpr int ai[4] = {1, 0, 1, 0}, bj[4] = {1, 2, 0, 1};
};
template <> struct Prods<32> {
    static constexpr int P = 3, n = 4;
    static constexpr int ai[4] = {2, 1, 1, 0}, bj[4] = {0, 1, 0, 1};
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
    int fp64_sum = 0;     // X = hi + lo and the alpha/beta epilogue in FP64, one rounding
    int grid_cus = 0;     // compute units the launch may use (0: all); host side only
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

// Output tiles that one workgroup of a persistent launch computes back to
// back: logical indices first, first + stride, ... (count of them) of a
// problem with tiles_m x tiles_n tiles, each mapped to its output tile as a
// one-tile-per-workgroup launch maps its workgroup index (XCD-aware remap,
// then 8 tile rows per group, column-major inside the group).
struct TileSeq {
    int first, stride, count, total, tiles_m, tiles_n;
    uint32_t inv_band, inv_last;   // udiv_inv of 8 tiles_n and of tiles_m % 8
};

// Division of uniform 32-bit values by a divisor fixed for the launch, in
// scalar registers (no floating-point reciprocal on the vector ALU): inv =
// floor((2^32 - 1) / d) makes mulhi(n, inv) equal to n / d or up to two less,
// which the two corrections fix.
__device__ __forceinline__ uint32_t udiv_inv(uint32_t d) { return d ? 0xFFFFFFFFu / d : 0u; }
__device__ __forceinline__ uint32_t udiv(uint32_t n, uint32_t d, uint32_t inv) {
    uint32_t q = __umulhi(n, inv);
    if (n - q * d >= d) ++q;
    if (n - q * d >= d) ++q;
    return q;
}

__device__ __forceinline__ void seq_init(TileSeq &q) {
    q.inv_band = udiv_inv(8u * (uint32_t)q.tiles_n);
    q.inv_last = udiv_inv((uint32_t)q.tiles_m & 7u);
}

__device__ __forceinline__ void seq_tile(const TileSeq &q, int k, int &tm, int &tn) {
    const int bid = q.first + k * q.stride;
    const int qq = q.total >> 3, r = q.total & 7;
    const int xcd = bid & 7, slot = bid >> 3;
    const int id = (xcd < r) ? xcd * (qq + 1) + slot : r * (qq + 1) + (xcd - r) * qq + slot;
    const int group = (int)udiv((uint32_t)id, 8u * (uint32_t)q.tiles_n, q.inv_band);
    const int first_m = group * 8;
    const int in_g = id - group * 8 * q.tiles_n;
    if (q.tiles_m - first_m >= 8) {
        tm = first_m + (in_g & 7);
        tn = in_g >> 3;
    } else {
        const uint32_t gsz = (uint32_t)(q.tiles_m - first_m);
        tn = (int)udiv((uint32_t)in_g, gsz, q.inv_last);
        tm = first_m + (in_g - tn * (int)gsz);
    }
}

// LDS bytes one tile call needs.
template <int V, int BM, int BN>
constexpr size_t tile_lds_bytes() {
    return 2ull * Prods<V>::P * (BM + BN) * LDK * sizeof(uint16_t);
}

// LDS row length (BF16) of the wave-specialised tile: 128-wide tiles use
// unpadded 64-byte rows with the permuted layout of swz_off, 64-wide tiles
// the padded 80-byte rows of the general tile.
template <int BM>
constexpr int fast_ldk() { return BM == 128 ? BK : LDK; }

// The wave-specialised tile additionally keeps, per helper thread, room for
// its 2*KPT FP32 values (rare exact re-split path; stride padded by one).
template <int V, int BM, int BN>
constexpr size_t fast_lds_bytes() {
    return 2ull * Prods<V>::P * (BM + BN) * fast_ldk<BM>() * sizeof(uint16_t) +
           256ull * (2 * (BM * 32 / 256) + 1) * sizeof(float);
}

// Element offset of (row n, k) in a plane of the 128-wide wave-specialised
// tile (rows of 32 BF16 = 64 bytes; n counts A rows, then B columns).  Row n
// sits in physical row n ^ ((n >> 2) & 1) and its 16-byte chunk k/8 at
// position (k/8) ^ ((n >> 1) & 3).  On gfx950 (64 banks of 4 bytes) this keeps
// three access patterns free of bank conflicts: the MFMA fragment reads
// (16-byte reads of rows n0 + lane%16, chunk lane/16), the helpers' 8-byte
// stores of A (two consecutive rows per 16 lanes) and their 8-byte stores of
// B (columns 4 apart, whose physical rows then alternate in parity).
__device__ __forceinline__ int swz_off(int n, int k) {
    return ((n ^ ((n >> 2) & 1)) << 5) + ((((k >> 3) ^ (n >> 1)) & 3) << 3) + (k & 7);
}

// A wave-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Buffer resource over a wave's C block at (r0, c0) (uniform), rows x cols
// of it inside C, the block spanning less than 2^31 bytes.
template <int TM, int TN>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t c_block_rsrc(const GemmParams &p, int64_t r0, int64_t c0,
                                                              int rows = TM * 16, int cols = TN * 16) {
    const int bytes = ((rows - 1) * (int)p.ldc + cols) * 4;
    return __builtin_amdgcn_make_buffer_rsrc((void *)(p.C + r0 * p.ldc + c0), (short)0, bytes, 0x00020000);
}

// Epilogue of one wave's block whose TM*16 rows span less than 2^31 bytes of
// C: straight-line code with no per-element branch.  Buffer loads and stores
// take the lane's part of the address in one VGPR and the element's (uniform)
// part in an SGPR, so the C values of CB bands are in flight together and the
// stores issue back to back; nothing waits for a store to complete.  MASK
// (blocks crossing the edge of C): the buffer covers C from the block's
// origin to its last element inside C, and an element outside C takes a
// lane offset beyond that range, so its load returns 0 and its store is
// dropped.  Same arithmetic as the general epilogue.
template <int TM, int TN, int CB, bool MASK = false, bool ONLY_BETA_F32 = false>
__device__ __forceinline__ void epilogue_block(const GemmParams &p, const bfx_f32x4 (&hi)[TM][TN],
                                               const bfx_f32x4 (&lo)[TM][TN], int64_t row0, int64_t col0,
                                               int kg, int r16) {
    const int ldc = (int)p.ldc;
    const int64_t r0 = row0, c0 = col0;   // uniform (scalar registers)
    int rows = TM * 16, cols = TN * 16;   // extent of the block inside C
    if constexpr (MASK) {
        if (p.M - r0 < rows) rows = (int)(p.M - r0);
        if (p.N - c0 < cols) cols = (int)(p.N - c0);
        if (rows <= 0 || cols <= 0) return;
    }
    const __amdgpu_buffer_rsrc_t rc = c_block_rsrc<TM, TN>(p, r0, c0, rows, cols);
    const int vo_ = (kg * 4 * ldc + r16) * 4;
    auto vo = [&](int i, int j, int e) {
        if constexpr (MASK)
            return (i * 16 + kg * 4 + e < rows && j * 16 + r16 < cols) ? vo_ : (int)0x80000000;
        else
            return vo_;
    };
    auto so = [&](int i, int j, int e) { return ((i * 16 + e) * ldc + j * 16) * 4; };
    const float alpha = p.alpha, beta = p.beta;
    // one straight-line body per case (uniform branches outside the loops)
    auto body = [&](auto f64c, auto beta0c) {
        constexpr bool F64 = decltype(f64c)::value, B0 = decltype(beta0c)::value;
#pragma unroll
        for (int i0 = 0; i0 < TM; i0 += CB) {
            float cv[CB][TN][4];
            if constexpr (!B0) {
#pragma unroll
                for (int ii = 0; ii < CB; ++ii)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            cv[ii][j][e] =
                                __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rc, vo(i0 + ii, j, e), so(i0 + ii, j, e), 0));
            }
#pragma unroll
            for (int ii = 0; ii < CB; ++ii)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float h = hi[i0 + ii][j][e], l = lo[i0 + ii][j][e];
                        float x;
                        if constexpr (B0)
                            x = F64 ? (float)((double)alpha * ((double)h + (double)l)) : alpha * (h + l);
                        else
                            x = F64 ? (float)fma((double)alpha, (double)h + (double)l, (double)beta * (double)cv[ii][j][e])
                                    : fmaf(alpha, h + l, beta * cv[ii][j][e]);
                        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rc, vo(i0 + ii, j, e), so(i0 + ii, j, e), 0);
                    }
        }
    };
    static_assert(TM % CB == 0, "bands per batch must divide the bands");
    using T = std::true_type;
    using F = std::false_type;
    if constexpr (ONLY_BETA_F32) {
        body(F{}, F{});   // the caller has beta != 0 and the FP32 sum
        return;
    }
    if (beta == 0.0f) {
        if (p.fp64_sum) body(T{}, T{});
        else body(F{}, T{});
    } else {
        if (p.fp64_sum) body(T{}, F{});
        else body(F{}, F{});
    }
}

// Epilogue of one MFMA wave's TM x TN block of 16 x 16 tiles.  Output layout
// of v_mfma_f32_16x16x32_bf16: lane holds column lane%16, rows 4*(lane/16) +
// 0..3 of each 16 x 16 tile.  X = hi + lo (the largest bin added last), then
// C = alpha X (beta == 0: C not read) or fma(alpha, X, beta C), or, for
// split-K, the hi and lo partial sums.  With fp64_sum (the "d" option of
// Sec. IV-A) X and the alpha/beta combination are formed in FP64 and rounded
// once.  With beta != 0 the C values of CB
// 16-row bands are all loaded before their first store, so those loads are
// in flight together instead of each waiting for the previous store.
template <int TM, int TN, int CB = TM>
__device__ __forceinline__ void tile_epilogue(const GemmParams &p, const bfx_f32x4 (&hi)[TM][TN],
                                              const bfx_f32x4 (&lo)[TM][TN], int64_t row0,
                                              int64_t col0, int kg, int r16, int64_t split) {
    auto row_of = [&](int i, int e) { return row0 + i * 16 + kg * 4 + e; };
    auto col_of = [&](int j) { return col0 + j * 16 + r16; };
    if (p.splits > 1) {
        const int64_t MN = p.M * p.N;
        float *base = p.partial + (split * 2) * MN;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = row_of(i, e), col = col_of(j);
                    if (row >= p.M || col >= p.N) continue;
                    base[row * p.N + col] = hi[i][j][e];
                    base[MN + row * p.N + col] = lo[i][j][e];
                }
        return;
    }
    // (row0, col0) is the same in every lane of the wave
    const int64_t ur0 = uniform_i64(row0), uc0 = uniform_i64(col0);
    if (((int64_t)(TM * 16 - 1) * p.ldc + TN * 16) * 4 < (int64_t(1) << 31)) {
        if (ur0 + TM * 16 <= p.M && uc0 + TN * 16 <= p.N) epilogue_block<TM, TN, CB>(p, hi, lo, ur0, uc0, kg, r16);
        else epilogue_block<TM, TN, CB, true>(p, hi, lo, ur0, uc0, kg, r16);
        return;
    }
    if (p.beta == 0.0f) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = row_of(i, e), col = col_of(j);
                    if (row >= p.M || col >= p.N) continue;
                    p.C[row * p.ldc + col] =
                        p.fp64_sum ? (float)((double)p.alpha * ((double)hi[i][j][e] + (double)lo[i][j][e]))
                                   : p.alpha * (hi[i][j][e] + lo[i][j][e]);
                }
        return;
    }
    // CB 16-row bands at a time: all their C values are loaded before the
    // first store, so that those loads are in flight together
    static_assert(TM % CB == 0, "bands per batch must divide the bands");
#pragma unroll
    for (int i0 = 0; i0 < TM; i0 += CB) {
        float cv[CB][TN][4];
#pragma unroll
        for (int ii = 0; ii < CB; ++ii)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = row_of(i0 + ii, e), col = col_of(j);
                    cv[ii][j][e] = (row < p.M && col < p.N) ? p.C[row * p.ldc + col] : 0.0f;
                }
#pragma unroll
        for (int ii = 0; ii < CB; ++ii)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t row = row_of(i0 + ii, e), col = col_of(j);
                    if (row >= p.M || col >= p.N) continue;
                    p.C[row * p.ldc + col] =
                        p.fp64_sum
                            ? (float)fma((double)p.alpha, (double)hi[i0 + ii][j][e] + (double)lo[i0 + ii][j][e],
                                         (double)p.beta * (double)cv[ii][j][e])
                            : fmaf(p.alpha, hi[i0 + ii][j][e] + lo[i0 + ii][j][e], p.beta * cv[ii][j][e]);
                }
    }
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

    tile_epilogue<TM, TN>(p, hi, lo, m0 + wm * TM * 16, n0 + wn * TN * 16, kg, r16, split);
}


// ---------------------------------------------------------------------------
// Fast path: BM x BN tile (128 x 128 or 64 x 64), 4 MFMA + 4 helper waves.
// Requirements: A and B rows 16-byte aligned (pointers 16-byte aligned, lda
// and ldb multiples of 4), K % 4 == 0, N % 4 == 0 and the K range of a split
// a multiple of 32.  M, N and K need
// not fill the tile: partial tiles are handled by clamped loads whose values
// are replaced by zeros and by a masked epilogue.  Differences from gemm_tile:
//   * loads: 16-byte buffer loads of A row segments and B row segments
//     (4 columns); every helper thread holds 4 consecutive k of BM/32 A rows
//     and 4 columns x BN/32 consecutive k of B, so every LDS store is an
//     8-byte store of 4 BF16 of one row (A) or one column (B); the 128-wide
//     tile uses the bank-conflict-free layout of swz_off, the 64-wide tile
//     padded 80-byte rows;
//   * global loads are issued three (128-wide tiles) or two (64-wide) K-steps
//     ahead, one register stage per step in flight;
//   * the split is branch-free (hardware RNE); the rare values for which it is
//     not exact (Inf/NaN, or a first term that rounds to Inf) are detected from
//     the first plane and the thread's values re-split exactly before its
//     register stage is reloaded.
// ---------------------------------------------------------------------------

// Issue order of one K-step's products (the lo products of Prods<V> grouped
// by B plane, largest plane first, then the hi product A0 B0) and the read
// group of each operand
// plane: group 0 = the planes of the first product, group 1 = the planes the
// second product adds, group 2 = the rest.  Reading in this order lets the
// first MFMAs of a step start after 5 fragment reads instead of waiting
// behind all of A's (measured 3-6% at 8192^3 x6), and spreading groups 1
// and 2 over the first two products' MFMAs another ~5%.
template <int V>
struct StepOrder {
    static constexpr int NPROD = Prods<V>::n + 1;
    int a[NPROD], b[NPROD];   // A and B plane of product k; product NPROD-1 is the hi product
    int ga[3], gb[3];         // read group of A plane pl and B plane pl
    constexpr StepOrder() : a(), b(), ga(), gb() {
        int k = 0;
        for (int jp = Prods<V>::P - 1; jp >= 0; --jp)
            for (int q = 0; q < Prods<V>::n; ++q)
                if (Prods<V>::bj[q] == jp) {
                    a[k] = Prods<V>::ai[q];
                    b[k] = jp;
                    ++k;
                }
        a[k] = 0;
        b[k] = 0;
        for (int pl = 0; pl < 3; ++pl) ga[pl] = gb[pl] = 2;
        ga[a[0]] = 0;
        gb[b[0]] = 0;
        if (NPROD > 1) {
            if (ga[a[1]] == 2) ga[a[1]] = 1;
            if (gb[b[1]] == 2) gb[b[1]] = 1;
        }
    }
};

// Scheduling request: R LDS reads spread over the MFMAs that follow, one
// read per M MFMAs (sched_group_barrier masks: 0x100 LDS read, 0x008 MFMA).
template <int R, int M, int ID>
__device__ __forceinline__ void interleave_reads() {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, ID);
        __builtin_amdgcn_sched_group_barrier(0x008, M, ID);
    }
}

// One K-step of an MFMA wave's TM x TN block of 16 x 16 tiles: fragments
// from the LDS planes at `base` (plane pl at pl * PLANE elements; A rows at
// aoff, B columns at boff) and the products in StepOrder's order (lo, then
// hi).  Read group 0 is read before the first product; group 1 is read
// while the first product's MFMAs issue and group 2 while the second's, one
// read between every few MFMAs (scheduling barriers hold the order).
template <int V, int TM, int TN, int PLANE>
__device__ __forceinline__ void mfma_step(const uint16_t *base, const int (&aoff)[TM], const int (&boff)[TN],
                                          bfx_f32x4 (&hi)[TM][TN], bfx_f32x4 (&lo)[TM][TN]) {
    constexpr int P = Prods<V>::P;
    constexpr int NPROD = StepOrder<V>::NPROD;
    constexpr StepOrder<V> O{};
    // reads in group g, and MFMAs per read when they are spread over one product
    constexpr auto reads = [](const StepOrder<V> &o, int g) {
        int r = 0;
        for (int pl = 0; pl < Prods<V>::P; ++pl) r += (o.gb[pl] == g ? TN : 0) + (o.ga[pl] == g ? TM : 0);
        return r;
    };
    constexpr int R1 = reads(O, 1), R2 = reads(O, 2);
    constexpr int M1 = R1 && TM * TN / R1 > 0 ? TM * TN / R1 : 1;
    constexpr int M2 = R2 && TM * TN / R2 > 0 ? TM * TN / R2 : 1;
    bfx_bf16x8 af[P][TM], bf[P][TN];
    auto read_group = [&](int g) {
#pragma unroll
        for (int pl = P - 1; pl >= 0; --pl)
            if (O.gb[pl] == g) {
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    bf[pl][j] = *reinterpret_cast<const bfx_bf16x8 *>(base + pl * PLANE + boff[j]);
            }
#pragma unroll
        for (int pl = 0; pl < P; ++pl)
            if (O.ga[pl] == g) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    af[pl][i] = *reinterpret_cast<const bfx_bf16x8 *>(base + pl * PLANE + aoff[i]);
            }
    };
    auto product = [&](int k) {
        bfx_f32x4 (&acc)[TM][TN] = (k == NPROD - 1) ? hi : lo;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[O.a[k]][i], bf[O.b[k]][j], acc[i][j], 0, 0, 0);
    };
    read_group(0);
    __builtin_amdgcn_sched_barrier(0);
    read_group(1);
    product(0);
    interleave_reads<R1, M1, 0>();
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (NPROD > 1) {
        read_group(2);
        product(1);
        interleave_reads<R2, M2, 1>();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 2; k < NPROD; ++k) product(k);
    }
}

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

// LDS row of B column n (0 <= n < BN) in the wave-specialised tile: inside
// every aligned group of 16 columns the low two bits are XORed with the group
// index, so that (a) the 16 columns an MFMA fragment read covers stay in 16
// distinct rows (conflict-free 16-byte reads, rows 80 bytes apart) and (b)
// the helpers' stores of column 4c + j (fixed j, c = 0..15) spread over 16
// row residues as well.
__device__ __forceinline__ int bcol_row(int n) { return (n & ~3) | ((n & 3) ^ ((n >> 4) & 3)); }

// Wave-specialised aligned tile: 512 threads.  Waves 0-3 (one per SIMD) only
// read BF16 fragments from LDS, run the MFMAs and write the epilogue; waves
// 4-7 (one per SIMD) only load FP32 tiles (2-3 K-steps ahead), split them and
// store the planes.  Every SIMD thus runs one wave of each kind and overlaps
// the split's VALU work with the other wave's matrix work.  Both kinds pass
// the same barrier once per K-step; the LDS planes are double-buffered.
// ECB: 16-row bands whose C values the epilogue loads together (0: all of
// them).  One band by default: more raise the kernel's register count, which
// cost the 8192^3 x6 launch 3%.
template <int V, int BM, int BN, int NST_ = 0, bool PERSIST = false, int ECB = 1, int EPI = 0>
__device__ __forceinline__ void gemm_tile_fast(const GemmParams &p, int64_t m0, int64_t n0,
                                               int64_t kb, int64_t ke, int64_t split,
                                               uint16_t *smem, const TileSeq *seq = nullptr) {
    using PR = Prods<V>;
    constexpr int P = PR::P;
    constexpr bool SWZ = BM == 128;                     // swz_off layout (else padded rows)
    constexpr int FLDK = fast_ldk<BM>();
    constexpr int PLANE = (BM + BN) * FLDK;
    constexpr int TM = BM / 32, TN = BN / 32;          // 16x16 tiles per MFMA wave (2 x 2 waves)
    constexpr int KPT = BM * BK / 256;                  // k values per helper thread
    constexpr int NST = NST_ ? NST_ : (BM == 128 ? 3 : 2);  // helper register stages
    static_assert(BM == BN && KPT % 8 == 0, "square tiles with >= 8 k values per helper thread");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int KT = (int)ceil_div(ke - kb, (int64_t)BK);
    // K-steps of the whole stream: one tile, or every tile of the sequence
    // (persistent launch: all tiles full, K a multiple of BK, no split-K)
    const int S = PERSIST ? seq->count * KT : KT;

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
        int boff[TN];   // B fragment offsets (elements) inside a plane
#pragma unroll
        for (int j = 0; j < TN; ++j)
            boff[j] = SWZ ? swz_off(BM + wn * (BN / 2) + j * 16 + r16, kg * 8)
                          : (BM + bcol_row(wn * (BN / 2) + j * 16 + r16)) * FLDK + kg * 8;
        int aoff[TM];   // A fragment offsets
#pragma unroll
        for (int i = 0; i < TM; ++i)
            aoff[i] = SWZ ? swz_off(wm * (BM / 2) + i * 16 + r16, kg * 8)
                          : (wm * (BM / 2) + i * 16 + r16) * FLDK + kg * 8;
        int tile_k = 0, step_in_tile = 0;   // persistent: tile and step within it
        // EPI == 1 (persistent, beta != 0, FP32 sum): the C values of a tile
        // are loaded at its first K-step and land while its K-steps run
        // (all of its address arithmetic in scalar registers: a vector
        // register written there would have to wait for the loads still in
        // flight into registers the allocator reuses)
        __amdgpu_buffer_rsrc_t crc;
        float cpre[EPI == 1 ? TM : 1][EPI == 1 ? TN : 1][4];
        const int cvo = (kg * 4 * (int)p.ldc + r16) * 4;
        auto cso = [&](int i, int j, int e) { return ((i * 16 + e) * (int)p.ldc + j * 16) * 4; };
        const int wm_u = __builtin_amdgcn_readfirstlane(wm), wn_u = __builtin_amdgcn_readfirstlane(wn);
        int next_tm = 0, next_tn = 0;   // EPI == 1: the next tile's indices
        if constexpr (PERSIST && EPI == 1) seq_tile(*seq, 0, next_tm, next_tn);
        for (int s = 0; s < S; ++s) {
            __syncthreads();  // buffer s&1 holds step s
            if constexpr (PERSIST && EPI == 1) {
                if (step_in_tile == 0) {
                    crc = c_block_rsrc<TM, TN>(p, (int64_t)next_tm * BM + wm_u * (BM / 2),
                                               (int64_t)next_tn * BN + wn_u * (BN / 2));
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                cpre[i][j][e] = __uint_as_float(
                                    __builtin_amdgcn_raw_buffer_load_b32(crc, cvo, cso(i, j, e), 0));
                }
            }
            mfma_step<V, TM, TN, PLANE>(smem + (s & 1) * P * PLANE, aoff, boff, hi, lo);
            if constexpr (PERSIST) {
                if (++step_in_tile == KT) {
                    // last K-step of this tile: its epilogue, overlapped with the
                    // helpers' loads and split of the next tile's first steps
                    // (every tile of a persistent launch is full)
                    if constexpr (EPI == 1) {
#pragma unroll
                        for (int i = 0; i < TM; ++i)
#pragma unroll
                            for (int j = 0; j < TN; ++j)
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const float x = fmaf(p.alpha, hi[i][j][e] + lo[i][j][e], p.beta * cpre[i][j][e]);
                                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), crc, cvo, cso(i, j, e), 0);
                                }
                        if (tile_k + 1 < seq->count) seq_tile(*seq, tile_k + 1, next_tm, next_tn);
                    } else {
                        // EPI == 2: beta != 0 and the FP32 sum only (one code
                        // path, so no wait for the stores at the next step)
                        int tm, tn;
                        seq_tile(*seq, tile_k, tm, tn);
                        epilogue_block<TM, TN, ECB ? ECB : TM, false, EPI == 2>(p, hi, lo,
                                                              uniform_i64((int64_t)tm * BM + wm * (BM / 2)),
                                                              uniform_i64((int64_t)tn * BN + wn * (BN / 2)), kg, r16);
                    }
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                            hi[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
                            lo[i][j] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
                        }
                    step_in_tile = 0;
                    ++tile_k;
                }
            }
        }
        __syncthreads();  // matches the helpers' final barrier
        if constexpr (!PERSIST)
            tile_epilogue<TM, TN, ECB ? ECB : TM>(p, hi, lo, m0 + wm * (BM / 2), n0 + wn * (BN / 2), kg, r16, split);
        return;
    }

    // ------------------------------ helper waves ------------------------------
    // A: eight lanes cover one row's 32 k (128 bytes) with 16-byte loads, so a
    //    wave's load touches 8 whole rows (8 cache lines); each thread holds
    //    4 consecutive k of AR = BM/32 rows (ar0, ar0+32, ...).
    // B: 16-byte loads of 4 columns; each thread holds 4 columns x RB =
    //    BN/32 consecutive k, stored per column as RB BF16 per plane.  For
    //    BN = 128 eight lanes cover 4 k rows of the same 4 columns and a
    //    wave's load touches 8 k rows x 128 bytes; for BN = 64 a half-wave
    //    covers all 64 columns of one k row (rows permuted by bcol_row).
    constexpr int AR = BM / 32;
    constexpr int RB = BN / 32;
    const int h = tid - 256;
    const int ar0 = h / 8, ac = h % 8;      // A: first row, 4-k chunk
    const int hl = h & 63, hw = h >> 6;     // helper lane, helper wave
    const int bc = SWZ ? h >> 3 : (hl & 15);                 // column group
    const int bkq = SWZ ? h & 7 : 4 * hw + (hl >> 4);        // k rows RB*bkq ..
    // Extent of this tile inside the matrices.  `full` (uniform) selects the
    // unmasked code; otherwise every load is clamped to an element inside the
    // tile's range and its value replaced by zero before the split.
    const int rows = (int)((p.M - m0 < BM) ? p.M - m0 : BM);
    const int cols = (int)((p.N - n0 < BN) ? p.N - n0 : BN);
    const int klen = (int)(ke - kb);
    const bool full = rows == BM && cols == BN && klen % BK == 0;
    const bool b_ok = 4 * bc < cols;        // N % 4 == 0: a vector is valid or not as a whole
    // Buffer resources over exactly the elements of this tile's A rows and B
    // columns (the range check is a second guard; no load leaves the range).
    const int lda = (int)p.lda, ldb = (int)p.ldb;
    __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.A + m0 * p.lda + kb), (short)0, ((rows - 1) * lda + klen) * 4, 0x00020000);
    __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.B + kb * p.ldb + n0), (short)0, ((klen - 1) * ldb + cols) * 4, 0x00020000);
    int rsrc_tile = -1;   // persistent: tile whose resources rA, rB hold (uniform)
    int voA[AR];                            // byte offset of (row, k = 0) of each A row
#pragma unroll
    for (int i = 0; i < AR; ++i) voA[i] = ((ar0 + 32 * i < rows) ? (ar0 + 32 * i) * lda : 0) * 4;
    const int voB = (RB * bkq * ldb + (b_ok ? 4 * bc : 0)) * 4;

    // One instantiation per case, so that each K loop is a single code path
    // and the compiler's wait counts on the register stages stay exact.
    auto helpers = [&](auto fullc) {
        constexpr bool FULL = decltype(fullc)::value;
        float ra[NST][KPT], rb[NST][KPT];   // ra[.][4i + j]: row ar0+32i, k = 4ac + j
        auto issue = [&](int st, int step) {
            if constexpr (FULL) {
                if constexpr (PERSIST) {
                    // step of the stream -> tile of the sequence and its K-step
                    const int tk = step / KT;
                    step -= tk * KT;
                    if (tk != rsrc_tile) {
                        int tm, tn;
                        seq_tile(*seq, tk, tm, tn);
                        rA = __builtin_amdgcn_make_buffer_rsrc((void *)(p.A + (int64_t)tm * BM * p.lda), (short)0,
                                                               ((BM - 1) * lda + klen) * 4, 0x00020000);
                        rB = __builtin_amdgcn_make_buffer_rsrc((void *)(p.B + (int64_t)tn * BN), (short)0,
                                                               ((klen - 1) * ldb + BN) * 4, 0x00020000);
                        rsrc_tile = tk;
                    }
                }
                // per-lane part (row, k chunk) in the VGPR offset, the step in
                // the uniform SGPR offset
                const int soA = step * BK * 4;
#pragma unroll
                for (int i = 0; i < AR; ++i) {
                    const bfx_f32x4 v = __builtin_bit_cast(
                        bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[i] + ac * 16, soA, 0));
                    ra[st][4 * i] = v[0]; ra[st][4 * i + 1] = v[1]; ra[st][4 * i + 2] = v[2]; ra[st][4 * i + 3] = v[3];
                }
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const bfx_f32x4 v = __builtin_bit_cast(
                        bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rB, voB, (step * BK + i) * ldb * 4, 0));
                    rb[st][4 * i] = v[0]; rb[st][4 * i + 1] = v[1]; rb[st][4 * i + 2] = v[2]; rb[st][4 * i + 3] = v[3];
                }
            } else {
                // k beyond the range: read k = 0 of the same row / column instead
                const int kA = step * BK + ac * 4;
                const int dA = (kA < klen) ? kA * 4 : 0;
#pragma unroll
                for (int i = 0; i < AR; ++i) {
                    const bfx_f32x4 v = __builtin_bit_cast(
                        bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rA, voA[i] + dA, 0, 0));
                    ra[st][4 * i] = v[0]; ra[st][4 * i + 1] = v[1]; ra[st][4 * i + 2] = v[2]; ra[st][4 * i + 3] = v[3];
                }
                const int kB = step * BK + RB * bkq;
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const int off = (kB + i < klen) ? voB + (step * BK + i) * ldb * 4 : voB - RB * bkq * ldb * 4;
                    const bfx_f32x4 v = __builtin_bit_cast(
                        bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rB, off, 0, 0));
                    rb[st][4 * i] = v[0]; rb[st][4 * i + 1] = v[1]; rb[st][4 * i + 2] = v[2]; rb[st][4 * i + 3] = v[3];
                }
            }
        };
        // Zeros for the values outside the tile (partial tiles only).
        auto mask = [&](int st, int step) {
            const bool kA_ok = step * BK + ac * 4 < klen;
            const int kB = step * BK + RB * bkq;
#pragma unroll
            for (int i = 0; i < AR; ++i) {
                const bool ok = kA_ok && ar0 + 32 * i < rows;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!ok) ra[st][4 * i + j] = 0.0f;
            }
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const bool ok = b_ok && kB + i < klen;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!ok) rb[st][4 * i + j] = 0.0f;
            }
        };
        auto stage = [&](int st, int buf, int step) {
            if constexpr (!FULL) mask(st, step);
            uint16_t *base = smem + buf * P * PLANE;
            uint32_t flag = 0, pa[3][KPT / 2], pb[3][KPT / 2];
            float bt[KPT];   // B values column by column: bt[RB * j + i] = k row i, column j
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < RB; ++i) bt[RB * j + i] = rb[st][4 * i + j];
            split_run_fast<P, KPT>(ra[st], pa, flag);
            split_run_fast<P, KPT>(bt, pb, flag);
#pragma unroll
            for (int pl = 0; pl < P; ++pl) {
                // A: 4 BF16 (8 bytes) per row
#pragma unroll
                for (int i = 0; i < AR; ++i)
                    *reinterpret_cast<uint2 *>(base + pl * PLANE +
                                               (SWZ ? swz_off(ar0 + 32 * i, ac * 4) : (ar0 + 32 * i) * FLDK + ac * 4)) =
                        make_uint2(pa[pl][2 * i], pa[pl][2 * i + 1]);
                // B: RB BF16 of each of the 4 columns
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint16_t *d = base + pl * PLANE +
                                  (SWZ ? swz_off(BM + 4 * bc + j, RB * bkq) : (BM + bcol_row(4 * bc + j)) * FLDK + RB * bkq);
                    if constexpr (RB == 4)
                        *reinterpret_cast<uint2 *>(d) = make_uint2(pb[pl][2 * j], pb[pl][2 * j + 1]);
                    else
                        *reinterpret_cast<uint32_t *>(d) = pb[pl][j];
                }
            }
            return flag;
        };
        // Rare path: split this thread's values exactly, one BF16 store at a time.
        // The values still sit in the register stage (masked); they go through a
        // per-thread LDS area so that the loop below indexes memory, not
        // registers.  It runs before the stage is reloaded and issues no global
        // load, so the prefetch accounting of the common path is unaffected.
        float *raw = reinterpret_cast<float *>(smem + 2 * P * PLANE) + h * (2 * KPT + 1);
        auto fixup = [&](int st, int buf) {
#pragma unroll
            for (int q = 0; q < KPT; ++q) {
                raw[q] = ra[st][q];
                raw[KPT + q] = rb[st][q];
            }
            uint16_t *base = smem + buf * P * PLANE;
#pragma unroll 1
            for (int e = 0; e < 2 * KPT; ++e) {
                const bool isA = e < KPT;
                const int q = e - KPT;   // B: q = 4 i + j, k row RB*bkq + i, column 4 bc + j
                const int row = isA ? ar0 + 32 * (e / 4) : BM + (SWZ ? 4 * bc + (q & 3) : bcol_row(4 * bc + (q & 3)));
                const int k = isA ? ac * 4 + (e % 4) : RB * bkq + (q >> 2);
                const int off = SWZ ? swz_off(row, k) : row * FLDK + k;
                uint32_t hh[3];
                split3_exact(raw[e], hh[0], hh[1], hh[2]);
#pragma unroll
                for (int pl = 0; pl < P; ++pl) base[pl * PLANE + off] = (uint16_t)hh[pl];
            }
        };
        // Barrier t starts MFMA step t (buffer t&1).  Between barriers t and
        // t+1 the helpers split step t+1 into buffer (t+1)&1 and reload the
        // register stage they just emptied with step t+1+NST: step s lives in
        // stage s % NST, loaded NST K-steps before it is split (NST = 3 for
        // 128-wide tiles, 2 for 64-wide ones, whose register budget allows two
        // workgroups per CU).  The steady-state loop has no conditional
        // loads, so every stage is consumed exactly NST-1 full stages behind
        // the newest loads.
        if (S > 0) {
            const int last = S - 1;
            auto lim = [&](int s) { return s < last ? s : last; };
            auto step_of = [&](int st, int s) {
                const uint32_t f = stage(st, s & 1, s);
                if (flag_bad(f)) fixup(st, s & 1);
            };
#pragma unroll
            for (int st = 0; st < NST; ++st) issue(st, lim(st));
            step_of(0, 0);
            issue(0, lim(NST));
            int t = 0;
            for (; t + NST < S; t += NST) {
#pragma unroll
                for (int u = 1; u <= NST; ++u) {
                    __syncthreads();
                    step_of(u % NST, t + u);
                    issue(u % NST, lim(t + u + NST));
                }
            }
            // t % NST == 0 and t + NST >= S: steps t+1 .. S-1 remain
#pragma unroll
            for (int u = 1; u < NST; ++u) {
                if (t + u < S) {
                    __syncthreads();
                    step_of(u, t + u);
                }
            }
            __syncthreads();    // barrier S-1
        }
    };
    if constexpr (PERSIST) helpers(std::true_type{});   // every tile of the stream is full
    else if (full) helpers(std::true_type{});
    else helpers(std::false_type{});
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Pre-split operands: the Sec. II-A split done once per operand, O(N^2) work
// against the O(N^3) products (the cost split of Sec. V).  split_blocks_kernel writes each operand's P BF16 planes
// as whole 128 x 32 blocks of 8 KiB, every block already in the swz_off order
// of the LDS staging above and zero-padded to whole blocks: block (r, s) of a
// plane holds rows 128 r .. 128 r + 127 of A (columns of B) and k = 32 s ..
// 32 s + 31, at element (r * KS + s) * 4096.  The tile below then fills its
// LDS with plain 16-byte direct-to-LDS loads (no registers, no split
// arithmetic on the critical path), and its MFMA waves run the instruction
// sequence of gemm_tile_fast on the same LDS image, so both give the same bits.
struct PlaneArgs {
    const uint16_t *A, *B;     // P planes each
    int64_t a_plane, b_plane;  // elements per plane
    int KS;                    // K blocks of 32 (K padded to a multiple of 32)
};

// LDS stages of the pre-split tile: as many 128 x 128 x 32 stages of P
// planes as fit the 160 KiB of a CU, at most four.
template <int V>
constexpr int planes_stages() { return Prods<V>::P == 3 ? 3 : 4; }

template <int V>
constexpr size_t planes_lds_bytes() {
    return (size_t)planes_stages<V>() * Prods<V>::P * 2 * 128 * BK * sizeof(uint16_t);
}

// s_waitcnt with only the vector-memory count limited (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// 512 threads.  Waves 0-3: as in gemm_tile_fast (fragments from LDS, MFMAs,
// epilogue).  Waves 4-7: direct-to-LDS loads, NS - 1 K-steps ahead into a
// ring of NS stages; wave 4 + h moves the 1 KiB pieces 2h and 2h + 1 of every
// 8 KiB block.  Barrier t starts MFMA step t (stage t % NS); right after it
// the loaders refill stage (t - 1) % NS, which step t - 1 has finished
// reading, with step t + NS - 1, and before barrier t + 1 they wait until
// step t + 1's pieces have landed.
template <int V>
__device__ __forceinline__ void gemm_tile_planes(const GemmParams &p, const PlaneArgs &q,
                                                 int64_t tm, int64_t tn, uint16_t *smem) {
    using PR = Prods<V>;
    constexpr int P = PR::P;
    constexpr int NS = planes_stages<V>();
    constexpr int BM = 128, BN = 128;
    constexpr int PLANE = (BM + BN) * BK;               // A block, then B block
    constexpr int TM = BM / 32, TN = BN / 32;
    constexpr int NI = 4 * P;                           // loads per K-step per loader wave
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int S = q.KS;

    if (wave < 4) {
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
        int boff[TN], aoff[TM];
#pragma unroll
        for (int j = 0; j < TN; ++j) boff[j] = swz_off(BM + wn * (BN / 2) + j * 16 + r16, kg * 8);
#pragma unroll
        for (int i = 0; i < TM; ++i) aoff[i] = swz_off(wm * (BM / 2) + i * 16 + r16, kg * 8);
        int st = 0;
        for (int s = 0; s < S; ++s) {
            __syncthreads();  // stage st holds step s
            mfma_step<V, TM, TN, PLANE>(smem + st * P * PLANE, aoff, boff, hi, lo);
            st = (st + 1 == NS) ? 0 : st + 1;
        }
        __syncthreads();  // matches the loaders' final barrier
        tile_epilogue<TM, TN, 1>(p, hi, lo, tm * BM + wm * (BM / 2), tn * BN + wn * (BN / 2), kg, r16, 0);
        return;
    }

    // ------------------------------ loader waves ------------------------------
    const int h = __builtin_amdgcn_readfirstlane(wave) - 4;   // uniform: LDS addresses in SGPRs
    __amdgpu_buffer_rsrc_t rs[2 * P];   // blocks of plane pl: A at 2 pl, B at 2 pl + 1
    const int range = q.KS * 8192;
#pragma unroll
    for (int pl = 0; pl < P; ++pl) {
        rs[2 * pl] = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(q.A + pl * q.a_plane + tm * q.KS * 4096), (short)0, range, 0x00020000);
        rs[2 * pl + 1] = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(q.B + pl * q.b_plane + tn * q.KS * 4096), (short)0, range, 0x00020000);
    }
    const int vo = lane * 16 + h * 2048;   // this lane's 16 bytes of piece 2h
    typedef __attribute__((address_space(3))) void *lds_ptr;
    auto issue = [&](int s, int stage) {
        uint16_t *d = smem + stage * P * PLANE + h * 1024;
#pragma unroll
        for (int b = 0; b < 2 * P; ++b)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs[b], (lds_ptr)(d + b * 4096 + jj * 512), 16,
                                                         vo + jj * 1024, s * 8192, 0, 0);
    };
    int ld_stage = 0;   // stage of the next step to load
    for (int s = 0; s < NS - 1 && s < S; ++s) {
        issue(s, ld_stage);
        ld_stage = (ld_stage + 1 == NS) ? 0 : ld_stage + 1;
    }
    for (int t = 0; t < S; ++t) {
        // steps t+1 .. t+NS-2 may still be in flight; step t must have landed
        const int ahead = (S - 1 - t < NS - 2) ? S - 1 - t : NS - 2;
        if constexpr (NS == 4) {
            if (ahead == 2) wait_vmcnt<2 * NI>();
            else if (ahead == 1) wait_vmcnt<NI>();
            else wait_vmcnt<0>();
        } else {
            if (ahead == 1) wait_vmcnt<NI>();
            else wait_vmcnt<0>();
        }
        // barrier t.  No fence: a workgroup release fence would wait for
        // every direct-to-LDS load in flight (vmcnt(0)), including the newer
        // steps'; the wait above already covers step t.
        __builtin_amdgcn_s_barrier();
        if (t + NS - 1 < S) {
            issue(t + NS - 1, ld_stage);
            ld_stage = (ld_stage + 1 == NS) ? 0 : ld_stage + 1;
        }
    }
    __builtin_amdgcn_s_barrier();  // matches the MFMA waves' final barrier
}

}  // namespace bfx
