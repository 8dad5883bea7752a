// Plain FP32 GEMM on the vector ALU (Sec. II-C): every output is one FP32 FMA
// chain over k in increasing order, starting at +0, so the result equals the
// textbook FP32 computation bit for bit.  The comparator for the split
// variants; written for the non-packed FP32 FMA path of gfx950.
//
// Tiling: 128 x 128 outputs per 256-thread workgroup, K-step 8, each thread
// owns an 8 x 8 register block made of four 4 x 4 quadrants (rows ty*4 and
// 64 + ty*4, columns tx*4 and 64 + tx*4) so that its LDS reads are 16-byte
// and bank-conflict free.  Tiles staged through double-buffered LDS, A stored
// k-major (transposed on the way in).
#include "common.hpp"

namespace bfx {

namespace {
constexpr int SBM = 128, SBN = 128, SBK = 8, SPAD = 4;

struct SgemmParams {
    int64_t M, N, K;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
    float alpha, beta;
    int vecA, vecB;
    int64_t k_per_split;  // K range of one split (multiple of SBK)
    int splits;           // 1: direct epilogue, else partial sums
    float *partial;       // [splits][M][N]
};
}  // namespace

__device__ __forceinline__ int64_t xcd_remap_s(int64_t bid, int64_t total) {
    const int64_t q = total / 8, r = total % 8;
    const int64_t xcd = bid % 8, slot = bid / 8;
    return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

__global__ void __launch_bounds__(256, 2) sgemm_kernel(SgemmParams p) {
    __shared__ __align__(16) float As[2][SBK][SBM + SPAD];
    __shared__ __align__(16) float Bs[2][SBK][SBN + SPAD];

    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int64_t tiles_m = ceil_div(p.M, SBM), tiles_n = ceil_div(p.N, SBN);
    const int64_t tiles = tiles_m * tiles_n;
    const int64_t id0 = xcd_remap_s(blockIdx.x, tiles * p.splits);
    const int64_t split = id0 / tiles;
    const int64_t id = id0 % tiles;
    const int64_t kb = split * p.k_per_split;
    const int64_t ke = (kb + p.k_per_split < p.K) ? kb + p.k_per_split : p.K;
    constexpr int GROUP = 8;
    const int64_t group = id / (GROUP * tiles_n);
    const int64_t first_m = group * GROUP;
    const int64_t gsz = (tiles_m - first_m < GROUP) ? tiles_m - first_m : GROUP;
    const int64_t in_g = id % (GROUP * tiles_n);
    const int64_t m0 = (first_m + in_g % gsz) * SBM;
    const int64_t n0 = (in_g / gsz) * SBN;

    // A tile 128 x 8: thread loads row tid/2, k (tid%2)*4 .. +3
    const int a_row = tid / 2, a_k = (tid % 2) * 4;
    // B tile 8 x 128: thread loads row tid/32, columns (tid%32)*4 .. +3
    const int b_row = tid / 32, b_col = (tid % 32) * 4;

    float ra[4], rb[4];
    auto load = [&](int64_t k0) {
        const int64_t gm = m0 + a_row, gk = k0 + a_k;
        const float *sa = p.A + gm * p.lda + gk;
        if (gm < p.M && gk + 4 <= ke && p.vecA) {
            const float4 v = *reinterpret_cast<const float4 *>(sa);
            ra[0] = v.x; ra[1] = v.y; ra[2] = v.z; ra[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) ra[j] = (gm < p.M && gk + j < ke) ? sa[j] : 0.0f;
        }
        const int64_t bk = k0 + b_row, bn = n0 + b_col;
        const float *sb = p.B + bk * p.ldb + bn;
        if (bk < ke && bn + 4 <= p.N && p.vecB) {
            const float4 v = *reinterpret_cast<const float4 *>(sb);
            rb[0] = v.x; rb[1] = v.y; rb[2] = v.z; rb[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) rb[j] = (bk < ke && bn + j < p.N) ? sb[j] : 0.0f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < 4; ++j) As[buf][a_k + j][a_row] = ra[j];
        *reinterpret_cast<float4 *>(&Bs[buf][b_row][b_col]) = make_float4(rb[0], rb[1], rb[2], rb[3]);
    };

    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0f;

    const int64_t KT = (ke > kb) ? ceil_div(ke - kb, SBK) : 0;
    if (KT > 0) {
        load(kb);
        store(0);
        __syncthreads();
        for (int64_t s = 0; s < KT; ++s) {
            const int cur = (int)(s & 1);
            if (s + 1 < KT) load(kb + (s + 1) * SBK);
#pragma unroll
            for (int k = 0; k < SBK; ++k) {
                const float4 a0 = *reinterpret_cast<const float4 *>(&As[cur][k][ty * 4]);
                const float4 a1 = *reinterpret_cast<const float4 *>(&As[cur][k][64 + ty * 4]);
                const float4 b0 = *reinterpret_cast<const float4 *>(&Bs[cur][k][tx * 4]);
                const float4 b1 = *reinterpret_cast<const float4 *>(&Bs[cur][k][64 + tx * 4]);
                const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                const float b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
            }
            if (s + 1 < KT) store(cur ^ 1);
            __syncthreads();
        }
    }

#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t row = m0 + (i < 4 ? ty * 4 + i : 64 + ty * 4 + (i - 4));
        if (row >= p.M) continue;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t col = n0 + (j < 4 ? tx * 4 + j : 64 + tx * 4 + (j - 4));
            if (col >= p.N) continue;
            if (p.splits > 1) {
                p.partial[(split * p.M + row) * p.N + col] = acc[i][j];
            } else {
                float *c = p.C + row * p.ldc + col;
                *c = (p.beta == 0.0f) ? p.alpha * acc[i][j] : fmaf(p.alpha, acc[i][j], p.beta * *c);
            }
        }
    }
}

// Fixed-order sum of the split partials, then the epilogue (deterministic):
// pass 1 (only when splits > SG) sums groups of SG consecutive splits in
// increasing order, pass 2 sums the group results (or the splits) in order.
constexpr int SG = 16;

__global__ void __launch_bounds__(256)
sgemm_group_kernel(const float *__restrict__ partial, int splits, int64_t MN,
                   float *__restrict__ group) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= MN) return;
    const int s0 = g * SG;
    const int s1 = (s0 + SG < splits) ? s0 + SG : splits;
    float v[SG];
#pragma unroll
    for (int q = 0; q < SG; ++q) v[q] = (s0 + q < s1) ? partial[(int64_t)(s0 + q) * MN + e] : 0.0f;
    float h = 0.0f;
#pragma unroll
    for (int q = 0; q < SG; ++q)
        if (s0 + q < s1) h += v[q];
    group[(int64_t)g * MN + e] = h;
}

__global__ void __launch_bounds__(256)
sgemm_final_kernel(const float *__restrict__ src, int count, int64_t M, int64_t N,
                   float alpha, float beta, float *C, int64_t ldc) {
    const int64_t MN = M * N;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= MN) return;
    float X = 0.0f;
#pragma unroll 8
    for (int s = 0; s < count; ++s) X += src[(int64_t)s * MN + e];
    const int64_t row = e / N, col = e % N;
    float *c = C + row * ldc + col;
    *c = (beta == 0.0f) ? alpha * X : fmaf(alpha, X, beta * *c);
}

static int sgemm_groups(int splits) { return splits > SG ? (int)ceil_div(splits, SG) : 0; }

// Same policy as the split GEMM: split K only when the output has too few
// tiles to fill the GPU and K is long.
static int sgemm_splits(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = ceil_div(M, SBM) * ceil_div(N, SBN);
    if (tiles >= 256 || K < 512) return 1;
    int64_t s = ceil_div(512, tiles);
    const int64_t max_s = K / 256;
    if (s > max_s) s = max_s;
    return s < 1 ? 1 : (int)s;
}

}  // namespace bfx

extern "C" size_t bfx_sgemm_ws_size(int64_t M, int64_t N, int64_t K) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    const int s = bfx::sgemm_splits(M, N, K);
    return s > 1 ? (size_t)(s + bfx::sgemm_groups(s)) * (size_t)M * (size_t)N * sizeof(float) : 0;
}

extern "C" int bfx_sgemm_fp32(int64_t M, int64_t N, int64_t K, float alpha,
                              const float *A, int64_t lda, const float *B, int64_t ldb,
                              float beta, float *C, int64_t ldc, void *ws, size_t ws_bytes,
                              void *stream) {
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (lda < (K > 1 ? K : 1)) return -6;
    if (ldb < (N > 1 ? N : 1)) return -8;
    if (ldc < (N > 1 ? N : 1)) return -11;
    if (M == 0 || N == 0) return BFX_OK;
    if (K > 0 && !A) return -5;
    if (K > 0 && !B) return -7;
    if (!C) return -10;
    bfx::SgemmParams p;
    p.M = M; p.N = N; p.K = K;
    p.A = A; p.lda = lda; p.B = B; p.ldb = ldb; p.C = C; p.ldc = ldc;
    p.alpha = alpha; p.beta = beta;
    p.vecA = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    p.vecB = ((uintptr_t)B % 16 == 0) && (ldb % 4 == 0);
    p.splits = bfx::sgemm_splits(M, N, K);
    p.k_per_split = bfx::ceil_div(bfx::ceil_div(K > 0 ? K : 1, p.splits), bfx::SBK) * bfx::SBK;
    p.splits = (int)bfx::ceil_div(K > 0 ? K : 1, p.k_per_split);
    p.partial = (float *)ws;
    const int groups = bfx::sgemm_groups(p.splits);
    if (p.splits > 1 && (size_t)(p.splits + groups) * M * N * sizeof(float) > ws_bytes) return -13;
    const int64_t blocks = bfx::ceil_div(M, bfx::SBM) * bfx::ceil_div(N, bfx::SBN) * p.splits;
    hipLaunchKernelGGL(bfx::sgemm_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, p);
    BFX_LAUNCH_CHECK("sgemm_kernel launch");
    if (p.splits > 1) {
        const unsigned rb = (unsigned)bfx::ceil_div(M * N, 256);
        const float *src = p.partial;
        int count = p.splits;
        if (groups > 0) {
            float *grp = p.partial + (size_t)p.splits * M * N;
            hipLaunchKernelGGL(bfx::sgemm_group_kernel, dim3(rb, (unsigned)groups), dim3(256), 0,
                               (hipStream_t)stream, p.partial, p.splits, M * N, grp);
            BFX_LAUNCH_CHECK("sgemm_group_kernel launch");
            src = grp;
            count = groups;
        }
        hipLaunchKernelGGL(bfx::sgemm_final_kernel, dim3(rb), dim3(256), 0, (hipStream_t)stream,
                           src, count, M, N, alpha, beta, C, ldc);
        BFX_LAUNCH_CHECK("sgemm_final_kernel launch");
    }
    return BFX_OK;
}
