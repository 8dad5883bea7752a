// Split-BF16 GEMM entry points (Sec. II-D, II-G, IV-A): one-problem launch,
// split-K for long inner dimensions with a deterministic fixed-order
// reduction, and the host-side tile / split policy.  The tile engine itself
// is in gemm_tile.hpp.
#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "gemm_tile.hpp"

namespace bfx {

template <int V, int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(WM *WN * 64, 1)
gemm_split_kernel(GemmParams p) {
    extern __shared__ __align__(16) uint16_t smem[];
    const int64_t tiles_m = ceil_div(p.M, BM), tiles_n = ceil_div(p.N, BN);
    const int64_t tiles = tiles_m * tiles_n;
    const int64_t total = tiles * p.splits;
    const int64_t id = xcd_remap(blockIdx.x, total);
    const int64_t split = id / tiles;
    const int64_t t = id % tiles;
    // grouped order: 8 tile rows per group, column-major inside the group
    constexpr int GROUP = 8;
    const int64_t group = t / (GROUP * tiles_n);
    const int64_t first_m = group * GROUP;
    const int64_t gsz = (tiles_m - first_m < GROUP) ? tiles_m - first_m : GROUP;
    const int64_t in_g = t % (GROUP * tiles_n);
    const int64_t m0 = (first_m + in_g % gsz) * BM;
    const int64_t n0 = (in_g / gsz) * BN;
    const int64_t kb = split * p.k_per_split;
    const int64_t ke = (kb + p.k_per_split < p.K) ? kb + p.k_per_split : p.K;
    gemm_tile<V, BM, BN, WM, WN>(p, m0, n0, kb, ke, split, smem);
}

// Output tile of tile index t (after the XCD-aware remap): groups of 4 tile
// columns, row-major inside the group, so that an XCD's workgroups sweep
// down the same B panels (measured at 8192^3 x6, average of 6 launches:
// 5.52-5.55 ms vs 5.60-5.82 grouping 4 tile rows and 5.73-5.81 grouping 8
// tile rows).
__device__ __forceinline__ void column_grouped_tile(int64_t t, int64_t tiles_m, int64_t tiles_n,
                                                    int64_t &tm, int64_t &tn) {
    constexpr int GROUP = 4;
    const int64_t group = t / (GROUP * tiles_m);
    const int64_t first_n = group * GROUP;
    const int64_t gsz = (tiles_n - first_n < GROUP) ? tiles_n - first_n : GROUP;
    const int64_t in_g = t % (GROUP * tiles_m);
    tn = first_n + in_g % gsz;
    tm = in_g / gsz;
}

// Wave-specialised tiles (see gemm_tile_fast), 512 threads: 4 MFMA + 4
// helper waves.
template <int V, int BM, int BN>
__global__ void __launch_bounds__(512, BM == 64 ? 2 : 1)
gemm_fast_kernel(GemmParams p) {
    extern __shared__ __align__(16) uint16_t smem[];
    const int64_t tiles_m = ceil_div(p.M, BM), tiles_n = ceil_div(p.N, BN);
    const int64_t tiles = tiles_m * tiles_n;
    const int64_t total = tiles * p.splits;
    const int64_t id = xcd_remap(blockIdx.x, total);
    const int64_t split = id / tiles;
    int64_t tm, tn;
    column_grouped_tile(id % tiles, tiles_m, tiles_n, tm, tn);
    const int64_t kb = split * p.k_per_split;
    const int64_t ke = (kb + p.k_per_split < p.K) ? kb + p.k_per_split : p.K;
    gemm_tile_fast<V, BM, BN>(p, tm * BM, tn * BN, kb, ke, split, smem);
}

// Split of one operand into the pre-split block layout of gemm_tile_planes
// (Sec. II-A, exact integer conversion for every element).  Each workgroup
// writes one block (r, s): rows 128 r .. of the operand (A rows; for TRANS,
// columns of a K x R row-major B) and k = 32 s .. 32 s + 31, zeros outside
// R x K.  A (TRANS false): each thread converts 16 consecutive k of
// one row (four 16-byte loads) and writes two 16-byte chunks per plane.
// B (TRANS true): the block is read with 16-byte loads along rows of B into
// LDS, then converted column by column like A.
template <int P, bool TRANS>
__device__ __forceinline__ void split_block(const float *__restrict__ X, int64_t ld, int64_t R, int64_t K,
                                            int KS, uint16_t *__restrict__ out, int64_t plane, bool vec,
                                            int64_t bid, float (*tile)[BK + 1]) {
    // A: consecutive block indices take consecutive k blocks of one row band
    // (rows read as contiguous runs); B: consecutive column bands of one k
    // band, so that together they read whole rows of B
    const int64_t RB = (R + 127) / 128;
    const int64_t r = TRANS ? bid % RB : bid / KS;
    const int64_t ks = TRANS ? bid / RB : bid % KS;
    const int t = threadIdx.x;
    uint16_t *blk = out + (r * KS + ks) * 4096;
    if constexpr (TRANS) {
        // 32 k rows x 128 columns through LDS: 16-byte loads along rows of B
        // (a wave reads two 512-byte rows per load), then each thread takes
        // 16 consecutive k of one column, as the A path does.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = t + 256 * i;
            const int kr = idx >> 5, c4 = idx & 31;
            const int64_t k = ks * BK + kr, col = r * 128 + 4 * c4;
            float f[4];
            if (vec && k < K && col + 4 <= R) {
                const float4 g = *reinterpret_cast<const float4 *>(X + k * ld + col);
                f[0] = g.x; f[1] = g.y; f[2] = g.z; f[3] = g.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) f[j] = (k < K && col + j < R) ? X[k * ld + col + j] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) tile[4 * c4 + j][kr] = f[j];
        }
        __syncthreads();
        const int n = t & 127, half = t >> 7;
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = tile[n][16 * half + i];
        __syncthreads();   // the tile is refilled by the workgroup's next block
        uint32_t w[3][8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint32_t x[3], y[3];
            split3_exact(v[2 * i], x[0], x[1], x[2]);
            split3_exact(v[2 * i + 1], y[0], y[1], y[2]);
#pragma unroll
            for (int pl = 0; pl < P; ++pl) w[pl][i] = x[pl] | (y[pl] << 16);
        }
#pragma unroll
        for (int pl = 0; pl < P; ++pl)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                *reinterpret_cast<uint4 *>(blk + pl * plane + swz_off(n, (2 * half + c) * 8)) =
                    make_uint4(w[pl][4 * c], w[pl][4 * c + 1], w[pl][4 * c + 2], w[pl][4 * c + 3]);
    } else {
        const int n = t >> 1, half = t & 1;
        const int64_t row = r * 128 + n;
        const int64_t k0 = ks * BK + 16 * half;
        float v[16];
        if (vec && row < R && k0 + 16 <= K) {
            const float4 *src = reinterpret_cast<const float4 *>(X + row * ld + k0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 f = src[i];
                v[4 * i] = f.x; v[4 * i + 1] = f.y; v[4 * i + 2] = f.z; v[4 * i + 3] = f.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t k = k0 + i;
                v[i] = (row < R && k < K) ? X[row * ld + k] : 0.0f;
            }
        }
        uint32_t w[3][8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint32_t x[3], y[3];
            split3_exact(v[2 * i], x[0], x[1], x[2]);
            split3_exact(v[2 * i + 1], y[0], y[1], y[2]);
#pragma unroll
            for (int pl = 0; pl < P; ++pl) w[pl][i] = x[pl] | (y[pl] << 16);
        }
#pragma unroll
        for (int pl = 0; pl < P; ++pl)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                *reinterpret_cast<uint4 *>(blk + pl * plane + swz_off(n, (2 * half + c) * 8)) =
                    make_uint4(w[pl][4 * c], w[pl][4 * c + 1], w[pl][4 * c + 2], w[pl][4 * c + 3]);
    }
}

template <int P, bool TRANS>
__global__ void __launch_bounds__(256)
split_blocks_kernel(const float *__restrict__ X, int64_t ld, int64_t R, int64_t K, int KS,
                    uint16_t *__restrict__ out, int64_t plane, bool vec) {
    __shared__ float tile[128][BK + 1];   // [column][k], odd stride: conflict-free column reads
    split_block<P, TRANS>(X, ld, R, K, KS, out, plane, vec, blockIdx.x, tile);
}

// Both operands of one product in one launch: workgroups [0, na) split one
// block of A each; the other gb workgroups split B's nb blocks with a grid
// stride (measured at 8192^2: A 144 us one block per workgroup, B 154 us
// over 4096 workgroups vs 166-184 us one block each; one launch saves the
// ~25 us between two).
template <int P>
__global__ void __launch_bounds__(256)
split_both_kernel(const float *__restrict__ A, int64_t lda, const float *__restrict__ B, int64_t ldb,
                  int64_t M, int64_t N, int64_t K, int KS, uint16_t *__restrict__ outA, int64_t planeA,
                  uint16_t *__restrict__ outB, int64_t planeB, bool vecA, bool vecB, int64_t na, int64_t nb) {
    __shared__ float tile[128][BK + 1];
    const int64_t b = blockIdx.x;
    if (b < na) {
        split_block<P, false>(A, lda, M, K, KS, outA, planeA, vecA, b, tile);
        return;
    }
    const int64_t gb = (int64_t)gridDim.x - na;
    for (int64_t q = b - na; q < nb; q += gb) split_block<P, true>(B, ldb, N, K, KS, outB, planeB, vecB, q, tile);
}

// GEMM on pre-split operands (see gemm_tile_planes): one 128 x 128 tile per
// workgroup, the tile order of gemm_fast_kernel.
template <int V>
__global__ void __launch_bounds__(512, 1)
gemm_planes_kernel(GemmParams p, PlaneArgs q) {
    extern __shared__ __align__(16) uint16_t smem[];
    const int64_t tiles_m = ceil_div(p.M, 128), tiles_n = ceil_div(p.N, 128);
    int64_t tm, tn;
    column_grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, tm, tn);
    gemm_tile_planes<V>(p, q, tm, tn, smem);
}

// Persistent wave-specialised launch for problems made of full 128 x 128
// tiles without split-K (computed as BM x BM tiles): workgroup b computes
// tiles b, b + grid, ... as one
// stream of K-steps, so that each tile's epilogue overlaps the helper waves'
// loads and split of the next tile's first K-steps (which a one-tile
// workgroup cannot overlap with anything: one such workgroup fills a CU).
template <int V, int BM = 128, int EPI = 0>
__global__ void __launch_bounds__(512, BM == 64 ? 2 : 1)
gemm_persist_kernel(GemmParams p, int total, int tiles_m, int tiles_n) {
    extern __shared__ __align__(16) uint16_t smem[];
    TileSeq seq;
    seq.first = (int)blockIdx.x;
    seq.stride = (int)gridDim.x;
    seq.count = (total - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x;
    seq.total = total;
    seq.tiles_m = tiles_m;
    seq.tiles_n = tiles_n;
    seq_init(seq);
    gemm_tile_fast<V, BM, BM, 0, true, 2, EPI>(p, 0, 0, 0, p.K, 0, smem, &seq);
}

// Fixed-order reduction of split-K partials, then the epilogue.  Two passes
// so that a long reduction over few outputs still spreads over many
// workgroups:
//   pass 1 (only when splits > SPLIT_GROUP): group g sums splits
//           g*SPLIT_GROUP .. in increasing order, hi and lo apart;
//   pass 2: the group sums (or the splits themselves) are added in increasing
//           order, X = hi + lo (the largest bin last), then the epilogue.
// The order depends only on the split count: deterministic.
constexpr int SPLIT_GROUP = 16;

__global__ void __launch_bounds__(256)
splitk_group_kernel(const float *__restrict__ partial, int splits, int64_t MN,
                    float *__restrict__ group) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= MN) return;
    const int s0 = g * SPLIT_GROUP;
    const int s1 = (s0 + SPLIT_GROUP < splits) ? s0 + SPLIT_GROUP : splits;
    float hv[SPLIT_GROUP], lv[SPLIT_GROUP];
#pragma unroll
    for (int q = 0; q < SPLIT_GROUP; ++q) {
        const bool in = s0 + q < s1;
        hv[q] = in ? partial[(int64_t)(2 * (s0 + q)) * MN + e] : 0.0f;
        lv[q] = in ? partial[(int64_t)(2 * (s0 + q) + 1) * MN + e] : 0.0f;
    }
    float h = 0.0f, l = 0.0f;
#pragma unroll
    for (int q = 0; q < SPLIT_GROUP; ++q) {
        if (s0 + q < s1) { h += hv[q]; l += lv[q]; }
    }
    group[(int64_t)(2 * g) * MN + e] = h;
    group[(int64_t)(2 * g + 1) * MN + e] = l;
}

__global__ void __launch_bounds__(256)
splitk_final_kernel(const float *__restrict__ src, int count, int64_t M, int64_t N,
                    float alpha, float beta, float *C, int64_t ldc, int fp64_sum) {
    const int64_t MN = M * N;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= MN) return;
    float h = 0.0f, l = 0.0f;
#pragma unroll 8
    for (int s = 0; s < count; ++s) {
        h += src[(int64_t)(2 * s) * MN + e];
        l += src[(int64_t)(2 * s + 1) * MN + e];
    }
    const int64_t row = e / N, col = e % N;
    float *c = C + row * ldc + col;
    if (fp64_sum) {
        const double X = (double)h + (double)l;
        *c = (beta == 0.0f) ? (float)((double)alpha * X) : (float)fma((double)alpha, X, (double)beta * (double)*c);
        return;
    }
    const float X = h + l;
    *c = (beta == 0.0f) ? alpha * X : fmaf(alpha, X, beta * *c);
}

static int split_groups(int splits) {
    return splits > SPLIT_GROUP ? (int)ceil_div(splits, SPLIT_GROUP) : 0;
}

// --------------------------------------------------------------------------
// Host side: tile choice and split-K policy.
// BFX_GEMM_GENERAL=1 in the environment disables the aligned fast path (used
// by tests to exercise the general engine on aligned shapes).
static const bool g_force_general = [] {
    const char *e = getenv("BFX_GEMM_GENERAL");
    return e && e[0] == '1';
}();
// --------------------------------------------------------------------------
template <int V, int BM, int BN, int WM, int WN>
static int launch_tiles(const GemmParams &p, hipStream_t s) {
    const size_t lds = tile_lds_bytes<V, BM, BN>();
    auto kern = gemm_split_kernel<V, BM, BN, WM, WN>;
    static bool attr_set = false;
    if (!attr_set) {
        BFX_HIP(hipFuncSetAttribute((const void *)kern,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int64_t blocks = ceil_div(p.M, BM) * ceil_div(p.N, BN) * p.splits;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WM * WN * 64), lds, s, p);
    BFX_LAUNCH_CHECK("gemm_split_kernel launch");
    return BFX_OK;
}

// Split-K is used when the output has too few tiles to fill the GPU and K is
// long: splits chosen so that about 4 workgroups run per CU, each covering at
// least 8 K-steps.
static int choose_splits(int64_t M, int64_t N, int64_t K, int BM, int BN) {
    const int64_t tiles = ceil_div(M, BM) * ceil_div(N, BN);
    const int64_t target = 512;
    if (tiles >= 256 || K < 16 * BK) return 1;
    int64_t s = ceil_div(target, tiles);
    const int64_t max_s = K / (8 * BK);
    if (s > max_s) s = max_s;
    if (s < 1) s = 1;
    return (int)s;
}

static void tile_for(int64_t M, int64_t N, int &BM, int &BN) {
    if (M <= 64 || N <= 64) { BM = 64; BN = 64; }
    else { BM = 128; BN = 128; }
}

size_t gemm_ws_bytes(int variant, int64_t M, int64_t N, int64_t K) {
    int BM, BN;
    tile_for(M, N, BM, BN);
    const int s = choose_splits(M, N, K, BM, BN);
    if (s <= 1) return 0;
    return (size_t)(s + split_groups(s)) * 2 * (size_t)M * (size_t)N * sizeof(float);
}

// Pre-split path (gemm_tile_planes): no split-K, at least 256 output tiles of
// 128 x 128 and K >= 512, where one O(N^2) split pass per operand is small
// against the products.  It runs when the caller's workspace holds the
// planes: P * (M + N) * K BF16 values, M and N padded to 128, K to 32.
// BFX_GEMM_PLANES=0 in the environment disables it (tests compare the two).
static const bool g_no_planes = [] {
    const char *e = getenv("BFX_GEMM_PLANES");
    return e && e[0] == '0';
}();

bool variant_valid(int v) {
    return v == 1 || v == 3 || v == 6 || v == 7 || v == 8 || v == 9 || v == 12 || v == 13 || v == 21 ||
           v == 23 || v == 31 || v == 32;
}

static int prods_p(int variant) {
    if (variant >= 10) return (variant / 10 > variant % 10) ? variant / 10 : variant % 10;
    return variant == 1 ? 1 : variant == 3 ? 2 : 3;
}

static bool planes_wanted(int64_t M, int64_t N, int64_t K) {
    const int64_t KS = ceil_div(K, BK);
    return !g_no_planes && ceil_div(M, 128) * ceil_div(N, 128) >= 256 && K >= 512 &&
           choose_splits(M, N, K, 128, 128) == 1 && KS * 8192 < (int64_t(1) << 31) &&
           ceil_div(M, 128) * ceil_div(N, 128) < (int64_t(1) << 31) &&
           ceil_div(M, 128) * KS < (int64_t(1) << 31) && ceil_div(N, 128) * KS < (int64_t(1) << 31);
}



static int64_t split_blocks_elems(int nterms, int64_t R, int64_t K);

static size_t planes_bytes(int variant, int64_t M, int64_t N, int64_t K) {
    const int P = prods_p(variant);
    return (size_t)(split_blocks_elems(P, M, K) + split_blocks_elems(P, N, K)) * sizeof(uint16_t);
}

static size_t gemm_ws_bytes_public(int variant, int64_t M, int64_t N, int64_t K) {
    const size_t s = gemm_ws_bytes(variant, M, N, K);
    const size_t pl = planes_wanted(M, N, K) ? planes_bytes(variant, M, N, K) : 0;
    return s > pl ? s : pl;
}

static int64_t split_blocks_elems(int nterms, int64_t R, int64_t K) {
    return (int64_t)nterms * ceil_div(R, 128) * ceil_div(K, BK) * 4096;
}

// One operand into nterms planes of the pre-split block layout.
static int launch_split_blocks(int nterms, bool trans, int64_t R, int64_t K, const float *X,
                               int64_t ld, uint16_t *out, hipStream_t s) {
    const int KS = (int)ceil_div(K, BK);
    const int64_t blocks = ceil_div(R, 128) * KS;
    const int64_t plane = blocks * 4096;
    const bool vec = ((uintptr_t)X % 16 == 0) && (ld % 4 == 0);
    const dim3 grid((unsigned)blocks), block(256);
#define BFX_SPLIT_BLOCKS(PP)                                                                       \
    if (trans)                                                                                     \
        hipLaunchKernelGGL((split_blocks_kernel<PP, true>), grid, block, 0, s, X, ld, R, K, KS, out, plane, vec); \
    else                                                                                           \
        hipLaunchKernelGGL((split_blocks_kernel<PP, false>), grid, block, 0, s, X, ld, R, K, KS, out, plane, vec);
    if (nterms == 1) { BFX_SPLIT_BLOCKS(1) }
    else if (nterms == 2) { BFX_SPLIT_BLOCKS(2) }
    else { BFX_SPLIT_BLOCKS(3) }
#undef BFX_SPLIT_BLOCKS
    BFX_LAUNCH_CHECK("split_blocks_kernel launch");
    return BFX_OK;
}

// The products on pre-split operands (p.A, p.B unused).
template <int V>
static int launch_gemm_blocks(const GemmParams &p, const uint16_t *Ab, const uint16_t *Bb, hipStream_t s) {
    const int KS = (int)ceil_div(p.K, BK);
    const int64_t rm = ceil_div(p.M, 128), rn = ceil_div(p.N, 128);
    PlaneArgs q;
    q.KS = KS;
    q.a_plane = rm * KS * 4096;
    q.b_plane = rn * KS * 4096;
    q.A = Ab;
    q.B = Bb;
    const size_t lds = planes_lds_bytes<V>();
    static bool attr_set = false;
    if (!attr_set) {
        BFX_HIP(hipFuncSetAttribute((const void *)gemm_planes_kernel<V>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    hipLaunchKernelGGL((gemm_planes_kernel<V>), dim3((unsigned)(rm * rn)), dim3(512), lds, s, p, q);
    BFX_LAUNCH_CHECK("gemm_planes_kernel launch");
    return BFX_OK;
}

static int gemm_blocks_dispatch(int variant, const GemmParams &p, const uint16_t *Ab, const uint16_t *Bb,
                                hipStream_t s) {
    switch (variant) {
        case 1: return launch_gemm_blocks<1>(p, Ab, Bb, s);
        case 3: return launch_gemm_blocks<3>(p, Ab, Bb, s);
        case 6: return launch_gemm_blocks<6>(p, Ab, Bb, s);
        case 7: return launch_gemm_blocks<7>(p, Ab, Bb, s);
        case 8: return launch_gemm_blocks<8>(p, Ab, Bb, s);
        case 9: return launch_gemm_blocks<9>(p, Ab, Bb, s);
        case 12: return launch_gemm_blocks<12>(p, Ab, Bb, s);
        case 13: return launch_gemm_blocks<13>(p, Ab, Bb, s);
        case 21: return launch_gemm_blocks<21>(p, Ab, Bb, s);
        case 23: return launch_gemm_blocks<23>(p, Ab, Bb, s);
        case 31: return launch_gemm_blocks<31>(p, Ab, Bb, s);
        case 32: return launch_gemm_blocks<32>(p, Ab, Bb, s);
        default: return -1;
    }
}

// Both operands split into the workspace (one launch), then the products.
static int launch_planes(int variant, const GemmParams &p, void *ws, hipStream_t s) {
    const int P = prods_p(variant);
    uint16_t *pa = (uint16_t *)ws;
    uint16_t *pb = pa + split_blocks_elems(P, p.M, p.K);
    const int KS = (int)ceil_div(p.K, BK);
    const int64_t na = ceil_div(p.M, 128) * KS, nb = ceil_div(p.N, 128) * KS;
    const int64_t gb = nb < 4096 ? nb : 4096;
    const bool vecA = ((uintptr_t)p.A % 16 == 0) && (p.lda % 4 == 0);
    const bool vecB = ((uintptr_t)p.B % 16 == 0) && (p.ldb % 4 == 0);
    const dim3 grid((unsigned)(na + gb)), block(256);
#define BFX_SPLIT_BOTH(PP)                                                                          \
    hipLaunchKernelGGL((split_both_kernel<PP>), grid, block, 0, s, p.A, p.lda, p.B, p.ldb, p.M, p.N, \
                       p.K, KS, pa, na * 4096, pb, nb * 4096, vecA, vecB, na, nb);
    if (P == 1) { BFX_SPLIT_BOTH(1) }
    else if (P == 2) { BFX_SPLIT_BOTH(2) }
    else { BFX_SPLIT_BOTH(3) }
#undef BFX_SPLIT_BOTH
    BFX_LAUNCH_CHECK("split_both_kernel launch");
    return gemm_blocks_dispatch(variant, p, pa, pb, s);
}

template <int V, int BM, int BN>
static int launch_fast(const GemmParams &p, hipStream_t s) {
    const size_t lds = fast_lds_bytes<V, BM, BN>();
    static bool attr_set = false;
    if (!attr_set) {
        BFX_HIP(hipFuncSetAttribute((const void *)gemm_fast_kernel<V, BM, BN>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int64_t blocks = ceil_div(p.M, BM) * ceil_div(p.N, BN) * p.splits;
    hipLaunchKernelGGL((gemm_fast_kernel<V, BM, BN>), dim3((unsigned)blocks), dim3(512), lds, s, p);
    BFX_LAUNCH_CHECK("gemm_fast_kernel launch");
    return BFX_OK;
}

// The wave-specialised path applies when A's and B's rows are 16-byte
// aligned, K and N are multiples of 4 (whole 16-byte vectors along k and n)
// and each split's K range is a multiple of 32.  Buffer offsets are 32-bit: BM rows of A and one split's K
// rows of B must each span less than 2^31 bytes.
// BFX_GEMM_PERSIST=0 in the environment disables the persistent launch (tests
// compare it with the one-tile-per-workgroup launch).
static const bool g_no_persist = [] {
    const char *e = getenv("BFX_GEMM_PERSIST");
    return e && e[0] == '0';
}();

static int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

template <int V, int BM, int EPI>
static int launch_persist_epi(const GemmParams &p, hipStream_t s) {
    const size_t lds = fast_lds_bytes<V, BM, BM>();
    static bool attr_set = false;
    if (!attr_set) {
        BFX_HIP(hipFuncSetAttribute((const void *)gemm_persist_kernel<V, BM, EPI>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    const int tiles_m = (int)(p.M / BM), tiles_n = (int)(p.N / BM);
    const int total = tiles_m * tiles_n;
    const int slots = (p.grid_cus > 0 ? p.grid_cus : device_cus()) * (BM == 64 ? 2 : 1);
    const int grid = total < slots ? total : slots;
    hipLaunchKernelGGL((gemm_persist_kernel<V, BM, EPI>), dim3((unsigned)grid), dim3(512), lds, s, p, total,
                       tiles_m, tiles_n);
    BFX_LAUNCH_CHECK("gemm_persist_kernel launch");
    return BFX_OK;
}

// beta != 0 with the FP32 sum (the LU's trailing updates): a kernel whose
// epilogue has that one case (64 x 64 tiles: each tile's C loaded at its first
// K-step, which the 128 x 128 tiles have no registers for); otherwise the
// kernel that selects the case at run time.
template <int V, int BM>
static int launch_persist(const GemmParams &p, hipStream_t s) {
    if (p.beta != 0.0f && !p.fp64_sum) return launch_persist_epi<V, BM, BM == 64 ? 1 : 2>(p, s);
    return launch_persist_epi<V, BM, 0>(p, s);
}

// Every tile full, one K range, and K short enough that the per-tile
// prologue and epilogue matter (measured at 8192 x 8192 x6: 5% faster at
// K = 512 and 2048, 10% at 16256 x 16256 x 128, no gain at K = 8192): the
// persistent launch applies.
static bool persist_ok(const GemmParams &p) {
    return !g_no_persist && p.splits == 1 && p.M % 128 == 0 && p.N % 128 == 0 && p.K % BK == 0 &&
           p.K <= 4096 && (p.M / 128) * (p.N / 128) < (int64_t(1) << 30) &&
           128 * p.ldc * 4 < (int64_t(1) << 31);   // a wave's C block in 32-bit buffer offsets
}

static bool fast_ok(const GemmParams &p, int BM, int BN) {
    (void)BN;
    return p.K % 4 == 0 && p.K > 0 && p.N % 4 == 0 && p.k_per_split % BK == 0 && p.vecA &&
           p.vecB && ((uintptr_t)p.C % 4 == 0) &&
           BM * p.lda * 4 < (int64_t(1) << 31) &&
           p.k_per_split * p.ldb * 4 < (int64_t(1) << 31);
}

template <int V>
static int dispatch_variant(GemmParams &p, int BM, int BN, hipStream_t s) {
    if (!g_force_general && fast_ok(p, BM, BN)) {
        if (BM == 128) {
            if (!persist_ok(p)) return launch_fast<V, 128, 128>(p, s);
            // K <= 128 (the LU's trailing updates): 64 x 64 tiles, two
            // workgroups per CU, measured 3-10% faster; longer K: 128 x 128
            return p.K <= 128 ? launch_persist<V, 64>(p, s) : launch_persist<V, 128>(p, s);
        }
        return launch_fast<V, 64, 64>(p, s);
    }
    if (BM == 64) return launch_tiles<V, 64, 64, 2, 2>(p, s);
    return launch_tiles<V, 128, 128, 2, 2>(p, s);
}

// Per-operand split counts: the general engine (and the pre-split products
// when the workspace holds the planes).
template <int V>
static int dispatch_general(GemmParams &p, int BM, hipStream_t s) {
    if (BM == 64) return launch_tiles<V, 64, 64, 2, 2>(p, s);
    return launch_tiles<V, 128, 128, 2, 2>(p, s);
}

int gemm_launch(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                const float *A, int64_t lda, const float *B, int64_t ldb,
                float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                hipStream_t stream, int flags, int grid_cus) {
    if (M == 0 || N == 0) return BFX_OK;
    int BM, BN;
    tile_for(M, N, BM, BN);
    GemmParams p;
    p.M = M; p.N = N; p.K = K;
    p.A = A; p.lda = lda; p.B = B; p.ldb = ldb; p.C = C; p.ldc = ldc;
    p.alpha = alpha; p.beta = beta;
    p.splits = choose_splits(M, N, K, BM, BN);
    p.k_per_split = ceil_div(ceil_div(K > 0 ? K : 1, p.splits), BK) * BK;
    p.splits = (int)ceil_div(K > 0 ? K : 1, p.k_per_split);
    p.partial = (float *)ws;
    p.vecA = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    p.vecB = ((uintptr_t)B % 16 == 0) && (ldb % 4 == 0);
    p.fp64_sum = (flags & BFX_GEMM_FP64_SUM) ? 1 : 0;
    p.grid_cus = grid_cus;
    const int groups = split_groups(p.splits);
    if (p.splits > 1 && (size_t)(p.splits + groups) * 2 * M * N * sizeof(float) > ws_bytes)
        return -14;
    if (p.splits == 1 && ws && (uintptr_t)ws % 16 == 0 && planes_wanted(M, N, K) &&
        ws_bytes >= planes_bytes(variant, M, N, K)) {
        return launch_planes(variant, p, ws, stream);
    }
    int rc;
    switch (variant) {
        case 1: rc = dispatch_variant<1>(p, BM, BN, stream); break;
        case 3: rc = dispatch_variant<3>(p, BM, BN, stream); break;
        case 6: rc = dispatch_variant<6>(p, BM, BN, stream); break;
        case 7: rc = dispatch_variant<7>(p, BM, BN, stream); break;
        case 8: rc = dispatch_variant<8>(p, BM, BN, stream); break;
        case 9: rc = dispatch_variant<9>(p, BM, BN, stream); break;
        case 12: rc = dispatch_general<12>(p, BM, stream); break;
        case 13: rc = dispatch_general<13>(p, BM, stream); break;
        case 21: rc = dispatch_general<21>(p, BM, stream); break;
        case 23: rc = dispatch_general<23>(p, BM, stream); break;
        case 31: rc = dispatch_general<31>(p, BM, stream); break;
        case 32: rc = dispatch_general<32>(p, BM, stream); break;
        default: return -1;
    }
    if (rc != BFX_OK || p.splits <= 1) return rc;
    const int64_t blocks = ceil_div(M * N, 256);
    const float *src = p.partial;
    int count = p.splits;
    if (groups > 0) {
        float *grp = p.partial + (size_t)p.splits * 2 * M * N;
        hipLaunchKernelGGL(splitk_group_kernel, dim3((unsigned)blocks, (unsigned)groups), dim3(256),
                           0, stream, p.partial, p.splits, M * N, grp);
        BFX_LAUNCH_CHECK("splitk_group_kernel launch");
        src = grp;
        count = groups;
    }
    hipLaunchKernelGGL(splitk_final_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       src, count, M, N, alpha, beta, C, ldc, p.fp64_sum);
    BFX_LAUNCH_CHECK("splitk_final_kernel launch");
    return BFX_OK;
}

}  // namespace bfx

extern "C" size_t bfx_gemm_ws_size(int variant, int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    return bfx::gemm_ws_bytes_public(variant, M, N, K);
}

extern "C" int bfx_gemm(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                        const float *A, int64_t lda, const float *B, int64_t ldb,
                        float beta, float *C, int64_t ldc, void *ws,
                        size_t ws_bytes, void *stream) {
    return bfx_gemm_ex(variant, 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, ws_bytes, stream);
}

extern "C" int bfx_gemm_ex(int variant, int flags, int64_t M, int64_t N, int64_t K, float alpha,
                           const float *A, int64_t lda, const float *B, int64_t ldb,
                           float beta, float *C, int64_t ldc, void *ws,
                           size_t ws_bytes, void *stream) {
    if (!bfx::variant_valid(variant)) return -1;
    if (flags & ~BFX_GEMM_FP64_SUM) return -2;
    if (M < 0) return -2;
    if (N < 0) return -3;
    if (K < 0) return -4;
    if (lda < (K > 1 ? K : 1)) return -7;
    if (ldb < (N > 1 ? N : 1)) return -9;
    if (ldc < (N > 1 ? N : 1)) return -12;
    if (M == 0 || N == 0) return BFX_OK;
    if (K > 0 && !A) return -6;
    if (K > 0 && !B) return -8;
    if (!C) return -11;
    return bfx::gemm_launch(variant, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws,
                            ws_bytes, (hipStream_t)stream, flags);
}

extern "C" size_t bfx_split_blocks_size(int nterms, int64_t R, int64_t K) {
    if (nterms < 1 || nterms > 3 || R <= 0 || K <= 0) return 0;
    return (size_t)bfx::split_blocks_elems(nterms, R, K) * sizeof(uint16_t);
}

extern "C" int bfx_split_blocks(int nterms, int trans, int64_t R, int64_t K, const float *X,
                                int64_t ld, uint16_t *out, size_t out_bytes, void *stream) {
    if (nterms < 1 || nterms > 3) return -1;
    if (trans != 0 && trans != 1) return -2;
    if (R < 0) return -3;
    if (K < 0) return -4;
    if (ld < (trans ? (R > 1 ? R : 1) : (K > 1 ? K : 1))) return -6;
    if (R == 0 || K == 0) return BFX_OK;
    if (!X) return -5;
    if (!out || (uintptr_t)out % 16 != 0) return -7;
    if (out_bytes < bfx_split_blocks_size(nterms, R, K)) return -8;
    if (bfx::ceil_div(K, bfx::BK) * 8192 >= (int64_t(1) << 31) ||
        bfx::ceil_div(R, 128) * bfx::ceil_div(K, bfx::BK) >= (int64_t(1) << 31))
        return -4;
    return bfx::launch_split_blocks(nterms, trans != 0, R, K, X, ld, out, (hipStream_t)stream);
}

extern "C" int bfx_gemm_blocks(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                               const uint16_t *Ab, const uint16_t *Bb, float beta, float *C,
                               int64_t ldc, void *stream) {
    if (!bfx::variant_valid(variant)) return -1;
    if (M < 0) return -2;
    if (N < 0) return -3;
    if (K < 0) return -4;
    if (ldc < (N > 1 ? N : 1)) return -10;
    if (M == 0 || N == 0) return BFX_OK;
    if (K == 0) {
        // no products: C = beta C (alpha * 0), through the general path
        return bfx::gemm_launch(variant, M, N, 0, alpha, nullptr, 1, nullptr, N, beta, C, ldc, nullptr, 0,
                                (hipStream_t)stream);
    }
    if (!Ab || (uintptr_t)Ab % 16 != 0) return -6;
    if (!Bb || (uintptr_t)Bb % 16 != 0) return -7;
    if (!C) return -9;
    const int64_t KS = bfx::ceil_div(K, bfx::BK);
    if (KS * 8192 >= (int64_t(1) << 31) || bfx::ceil_div(M, 128) * bfx::ceil_div(N, 128) >= (int64_t(1) << 31))
        return -4;
    bfx::GemmParams p = {};
    p.M = M; p.N = N; p.K = K;
    p.C = C; p.ldc = ldc;
    p.alpha = alpha; p.beta = beta;
    p.splits = 1;
    p.k_per_split = KS * bfx::BK;
    return bfx::gemm_blocks_dispatch(variant, p, Ab, Bb, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Allocation-free variant of bfx_gemm for callers that cannot allocate device
// memory.  Its workspace is `scratch`, a file-scope device array that every
// GPU the library runs on holds for the life of the process.  In host code
// the array's name is only a host-side stand-in: the device address is taken
// once per device with hipGetSymbolAddress and only that address is used.
// ---------------------------------------------------------------------------
namespace bfx {
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with the device current) and kept.
int scratch_address(void **out) {
    int dev = 0;
    BFX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("bfx_gemm_noalloc: device index beyond the supported range");
        return BFX_E_INTERNAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        BFX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("bfx_gemm_noalloc: hipGetSymbolAddress returned no address");
            return BFX_E_INTERNAL;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BFX_OK;
}
}  // namespace
}  // namespace bfx

extern "C" size_t bfx_gemm_noalloc_scratch_bytes(void) { return bfx::NOALLOC_SCRATCH_BYTES; }

extern "C" int bfx_gemm_noalloc(int variant, int64_t M, int64_t N, int64_t K, float alpha,
                                const float *A, int64_t lda, const float *B, int64_t ldb,
                                float beta, float *C, int64_t ldc, void *stream) {
    if (!bfx::variant_valid(variant)) return -1;
    if (M < 0) return -2;
    if (N < 0) return -3;
    if (K < 0) return -4;
    if (lda < (K > 1 ? K : 1)) return -7;
    if (ldb < (N > 1 ? N : 1)) return -9;
    if (ldc < (N > 1 ? N : 1)) return -12;
    if (M == 0 || N == 0) return BFX_OK;
    if (K > 0 && !A) return -6;
    if (K > 0 && !B) return -8;
    if (!C) return -11;
    // split-K partial sums are the only workspace the product cannot do without
    const size_t need = bfx::gemm_ws_bytes(variant, M, N, K);
    if (need > bfx::NOALLOC_SCRATCH_BYTES) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "bfx_gemm_noalloc: this shape needs %zu bytes of split-K scratch, "
                      "beyond the fixed maximum of %zu bytes",
                      need, bfx::NOALLOC_SCRATCH_BYTES);
        bfx::set_error(buf);
        return BFX_E_WORKSPACE;
    }
    void *ptr = nullptr;
    const int rc = bfx::scratch_address(&ptr);
    if (rc) return rc;
    return bfx::gemm_launch(variant, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ptr,
                            bfx::NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}
