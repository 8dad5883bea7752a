// Many independent dense solves A x = b (n <= 1024) in one persistent,
// graph-captured launch: split-BF16 blocked LU (Sec. I, IV-A) followed by
// FP64-residual iterative refinement (Sec. III), one workgroup per problem.
//
// Per problem, inside one 256-thread workgroup:
//   LU     panels of 32 columns held in LDS (pivot search by wave shuffles and
//          LDS, swap, divide, rank-1 update), interchanges on the other
//          columns, TRSM with L11 in LDS, and the trailing update
//          A22 -= L21 U12 through the split-GEMM tile engine (alpha = -1,
//          beta = 1, 64 x 64 tiles, one K-step of 32);
//   IR     |A|_inf and |b|_inf, the permutation from ipiv, then
//          x0 = LUsolve32(b) and refinement steps with an FP64 residual (one
//          wave per row) and FP32 triangular solves in 64-row blocks (the
//          diagonal block in LDS, solved by one wave).
// Problems are taken from a work counter in descending n (longest first);
// every workgroup loops until the list is exhausted.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "gemm_tile.hpp"

namespace bfx {

namespace {
constexpr int SNB = 32;          // panel width
constexpr int SLD = SNB + 1;     // LDS stride of a panel row
constexpr int SMAXN = 1024;      // largest n
constexpr int STB = 64;          // triangular-solve block
constexpr unsigned SOLVE_LDS = SMAXN * SLD * 4;   // panel; the other phases fit inside

struct SolveItem {
    int64_t n;
    const float *A;
    int64_t lda;
    const double *b;
    double *x;
    float *LU;        // n x n, leading dimension n
    int32_t *ipiv;
    bfx_ir_result *res;
    int32_t *info;
};
}  // namespace

__device__ __forceinline__ void argmax_better(float &v, int &i, float v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// Block-wide reductions for 256 threads (4 waves); every thread gets the result.
__device__ __forceinline__ void block_argmax(float &v, int &i, float *sv, int *si) {
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_xor(v, off);
        const int i2 = __shfl_xor(i, off);
        argmax_better(v, i, v2, i2);
    }
    if ((threadIdx.x & 63) == 0) { sv[threadIdx.x >> 6] = v; si[threadIdx.x >> 6] = i; }
    __syncthreads();
    v = sv[0];
    i = si[0];
    for (int k = 1; k < 4; ++k) argmax_better(v, i, sv[k], si[k]);
    __syncthreads();
}

__device__ __forceinline__ double block_max_d(double v, double *sd) {
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        if (o > v || o != o) v = o;
    }
    if ((threadIdx.x & 63) == 0) sd[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = sd[0];
    for (int k = 1; k < 4; ++k)
        if (sd[k] > m || sd[k] != sd[k]) m = sd[k];
    __syncthreads();
    return m;
}

// In-place FP32 solve of (L or U) y = y with y in LDS, factors in global LU.
template <bool LOWER>
__device__ void block_trsv(const float *LU, int n, float *y, float *D) {
    const int t = threadIdx.x, lane = t & 63;
    const int nblk = (n + STB - 1) / STB;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = LOWER ? bb : nblk - 1 - bb;
        const int k0 = blk * STB;
        const int rows = (n - k0 < STB) ? n - k0 : STB;
        for (int e = t; e < STB * STB; e += 256) {
            const int i = e / STB, c = e % STB;
            D[i * (STB + 1) + c] = (i < rows && c < rows) ? LU[(int64_t)(k0 + i) * n + k0 + c] : 0.0f;
        }
        __syncthreads();
        if (t < 64) {
            float v = (lane < rows) ? y[k0 + lane] : 0.0f;
            if (LOWER) {
                for (int c = 0; c < rows; ++c) {
                    const float yc = __shfl(v, c);
                    if (lane > c) v = fmaf(-D[lane * (STB + 1) + c], yc, v);
                }
            } else {
                for (int c = rows - 1; c >= 0; --c) {
                    if (lane == c) v = v / D[c * (STB + 1) + c];
                    const float yc = __shfl(v, c);
                    if (lane < c) v = fmaf(-D[lane * (STB + 1) + c], yc, v);
                }
            }
            if (lane < rows) y[k0 + lane] = v;
        }
        __syncthreads();
        // update the rows not yet solved with this block's solution
        const int lo = LOWER ? k0 + rows : 0, hi = LOWER ? n : k0;
        for (int i = lo + t; i < hi; i += 256) {
            const float *row = LU + (int64_t)i * n + k0;
            float acc = 0.0f;
            for (int c = 0; c < rows; ++c) acc = fmaf(row[c], y[k0 + c], acc);
            y[i] -= acc;
        }
        __syncthreads();
    }
}

template <int V>
__device__ void solve_one(const SolveItem &it, double tol, int max_iter, uint16_t *smem) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n = (int)it.n;
    float *LU = it.LU;
    __shared__ float s_v[4];
    __shared__ int s_i[4];
    __shared__ double s_d[4];

    // ---- copy A into the factor storage
    for (int64_t e = t; e < (int64_t)n * n; e += 256) {
        const int64_t r = e / n, c = e % n;
        LU[e] = it.A[r * it.lda + c];
    }
    if (t == 0) *it.info = 0;
    __syncthreads();

    // ---- blocked LU
    for (int j = 0; j < n; j += SNB) {
        const int jb = (n - j < SNB) ? n - j : SNB;
        const int m = n - j;
        float *P = reinterpret_cast<float *>(smem);
        for (int e = t; e < m * jb; e += 256) {
            const int r = e / jb, q = e % jb;
            P[r * SLD + q] = LU[(int64_t)(j + r) * n + j + q];
        }
        __syncthreads();
        for (int c = 0; c < jb; ++c) {
            float bv = -1.0f;
            int bi = INT_MAX;
            for (int r = c + t; r < m; r += 256) {
                float v = fabsf(P[r * SLD + c]);
                if (!(v == v)) v = INFINITY;
                argmax_better(bv, bi, v, r);
            }
            block_argmax(bv, bi, s_v, s_i);
            const int p = bi;
            if (t == 0) {
                it.ipiv[j + c] = j + p;
                if (P[p * SLD + c] == 0.0f && *it.info == 0) *it.info = j + c + 1;
            }
            if (p != c)
                for (int q = t; q < jb; q += 256) {
                    const float x = P[c * SLD + q];
                    P[c * SLD + q] = P[p * SLD + q];
                    P[p * SLD + q] = x;
                }
            __syncthreads();
            const float piv = P[c * SLD + c];
            for (int r = c + 1 + t; r < m; r += 256) {
                float l = P[r * SLD + c];
                if (piv != 0.0f) l = l / piv;
                P[r * SLD + c] = l;
                for (int q = c + 1; q < jb; ++q) P[r * SLD + q] = fmaf(-l, P[c * SLD + q], P[r * SLD + q]);
            }
            __syncthreads();
        }
        for (int e = t; e < m * jb; e += 256) {
            const int r = e / jb, q = e % jb;
            LU[(int64_t)(j + r) * n + j + q] = P[r * SLD + q];
        }
        __syncthreads();
        for (int col = t; col < n - jb; col += 256) {
            const int cc = col < j ? col : col + jb;
            for (int i = 0; i < jb; ++i) {
                const int r = j + i, p = it.ipiv[r];
                if (p != r) {
                    const float x = LU[(int64_t)r * n + cc];
                    LU[(int64_t)r * n + cc] = LU[(int64_t)p * n + cc];
                    LU[(int64_t)p * n + cc] = x;
                }
            }
        }
        __syncthreads();
        const int rest = n - j - jb;
        if (rest <= 0) continue;
        // U12 = L11^{-1} A12 in LDS: each thread solves its own columns in
        // row order (one FMA chain per entry in increasing p).
        {
            float *L = reinterpret_cast<float *>(smem);
            float *X = L + SNB * SNB;
            const int XLD = rest + 1;
            for (int e = t; e < SNB * SNB; e += 256) {
                const int i = e / SNB, p = e % SNB;
                L[e] = (i < jb && p < i) ? LU[(int64_t)(j + i) * n + j + p] : 0.0f;
            }
            for (int e = t; e < jb * rest; e += 256) {
                const int i = e / rest, c = e % rest;
                X[i * XLD + c] = LU[(int64_t)(j + i) * n + j + jb + c];
            }
            __syncthreads();
            for (int c = t; c < rest; c += 256)
                for (int i = 1; i < jb; ++i) {
                    float s = X[i * XLD + c];
                    for (int p = 0; p < i; ++p) s = fmaf(-L[i * SNB + p], X[p * XLD + c], s);
                    X[i * XLD + c] = s;
                }
            __syncthreads();
            for (int e = t; e < jb * rest; e += 256) {
                const int i = e / rest, c = e % rest;
                LU[(int64_t)(j + i) * n + j + jb + c] = X[i * XLD + c];
            }
            __syncthreads();
        }
        GemmParams gp;
        gp.M = rest; gp.N = rest; gp.K = jb;
        gp.A = LU + (int64_t)(j + jb) * n + j; gp.lda = n;
        gp.B = LU + (int64_t)j * n + j + jb; gp.ldb = n;
        gp.C = LU + (int64_t)(j + jb) * n + j + jb; gp.ldc = n;
        gp.alpha = -1.0f; gp.beta = 1.0f;
        gp.k_per_split = jb; gp.splits = 1; gp.partial = nullptr;
        gp.vecA = (n % 4 == 0) && (j % 4 == 0) && (((uintptr_t)LU) % 16 == 0);
        gp.vecB = (n % 4 == 0) && ((j + jb) % 4 == 0) && (((uintptr_t)LU) % 16 == 0);
        const int tiles = (rest + 63) / 64;
        for (int tm = 0; tm < tiles; ++tm)
            for (int tn = 0; tn < tiles; ++tn)
                gemm_tile<V, 64, 64, 2, 2>(gp, (int64_t)tm * 64, (int64_t)tn * 64, 0, jb, 0, smem);
        __syncthreads();
    }

    // ---- iterative refinement (Sec. III)
    float *y = reinterpret_cast<float *>(smem);                  // n floats
    double *r = reinterpret_cast<double *>(smem + 2 * SMAXN);    // n doubles (byte offset 4096)
    int32_t *perm = reinterpret_cast<int32_t *>(smem + 6 * SMAXN);  // n ints (byte offset 12288)
    float *D = reinterpret_cast<float *>(smem + 8 * SMAXN);      // 64 x 65 (byte offset 16384)
    const float *A = it.A;
    // norms
    double rowmax = 0.0;
    for (int row = wave; row < n; row += 4) {
        double s = 0.0;
        for (int c = lane; c < n; c += 64) s += fabs((double)A[(int64_t)row * it.lda + c]);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (s > rowmax) rowmax = s;
    }
    const double normA = block_max_d(rowmax, s_d);
    double bm = 0.0;
    for (int i = t; i < n; i += 256) {
        const double a = fabs(it.b[i]);
        if (a > bm || a != a) bm = a;
    }
    const double normb = block_max_d(bm, s_d);
    for (int i = t; i < n; i += 256) perm[i] = i;
    __syncthreads();
    if (t == 0)
        for (int i = 0; i < n; ++i) {
            const int p = it.ipiv[i];
            if (p != i) { const int q = perm[i]; perm[i] = perm[p]; perm[p] = q; }
        }
    __syncthreads();
    for (int i = t; i < n; i += 256) y[i] = (float)it.b[perm[i]];
    __syncthreads();
    block_trsv<true>(LU, n, y, D);
    block_trsv<false>(LU, n, y, D);
    for (int i = t; i < n; i += 256) it.x[i] = (double)y[i];
    __syncthreads();

    int iters = 0, rises = 0, status = 1;
    double eta = 0.0, prev_eta = INFINITY;
    for (;;) {
        double rl = 0.0;
        for (int row = wave; row < n; row += 4) {
            double s = 0.0;
            for (int c = lane; c < n; c += 64) s = fma((double)A[(int64_t)row * it.lda + c], it.x[c], s);
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            const double ri = it.b[row] - s;
            if (lane == 0) r[row] = ri;
            const double a = fabs(ri);
            if (a > rl || a != a) rl = a;
        }
        const double rn = block_max_d(rl, s_d);
        double xl = 0.0;
        for (int i = t; i < n; i += 256) {
            const double a = fabs(it.x[i]);
            if (a > xl || a != a) xl = a;
        }
        const double xn = block_max_d(xl, s_d);
        const double den = normA * xn + normb;
        eta = den > 0.0 ? rn / den : rn;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        if (!(eta <= INFINITY)) { status = 3; break; }   // NaN
        if (eta == INFINITY) { status = 3; break; }
        if (eta <= tol) { status = 0; break; }
        if (iters >= max_iter) { status = 1; break; }
        if (rises >= 2) { status = 2; break; }
        for (int i = t; i < n; i += 256) y[i] = (float)(r[perm[i]] / rn);
        __syncthreads();
        block_trsv<true>(LU, n, y, D);
        block_trsv<false>(LU, n, y, D);
        for (int i = t; i < n; i += 256) it.x[i] = fma(rn, (double)y[i], it.x[i]);
        __syncthreads();
        ++iters;
    }
    if (t == 0) {
        it.res->iters = iters;
        it.res->status = status;
        it.res->eta = eta;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(64) solve_zero_counter(uint32_t *c) {
    if (threadIdx.x == 0) *c = 0u;
}

template <int V>
__global__ void __launch_bounds__(256, 1)
persistent_solve_kernel(const SolveItem *__restrict__ items, int64_t count, uint32_t *counter,
                        double tol, int max_iter) {
    extern __shared__ __align__(16) uint16_t smem[];
    __shared__ int64_t s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
        solve_one<V>(items[idx], tol, max_iter, smem);
    }
}

}  // namespace bfx

struct bfx_solve_plan {
    int variant = 6;
    int64_t count = 0;
    bfx_ir_opts opts = {1e-14, 30, 0};
    std::vector<bfx_solve_desc> h_desc;
    std::vector<int64_t> lu_off, piv_off;   // host copies of per-problem offsets
    bfx::SolveItem *d_items = nullptr;
    float *d_lu = nullptr;
    int32_t *d_ipiv = nullptr;
    bfx_ir_result *d_res = nullptr;
    int32_t *d_info = nullptr;
    uint32_t *d_counter = nullptr;
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    int grid = 0;
    const void *kernel = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace bfx {
namespace {
void solve_plan_free(bfx_solve_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_lu) (void)hipFree(p->d_lu);
    if (p->d_ipiv) (void)hipFree(p->d_ipiv);
    if (p->d_res) (void)hipFree(p->d_res);
    if (p->d_info) (void)hipFree(p->d_info);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_ws) (void)hipFree(p->d_ws);
    delete p;
}
template <int V>
const void *solve_kernel_for() { return (const void *)persistent_solve_kernel<V>; }
}  // namespace
}  // namespace bfx

extern "C" int bfx_lu_ir_batched_plan_create(int variant, int64_t count, const bfx_solve_desc *descs,
                                             const bfx_ir_opts *opts, bfx_solve_plan **out) {
    using namespace bfx;
    if (variant != 1 && variant != 3 && variant != 6 && variant != 9) return -1;
    if (count < 0) return -2;
    if (count > 0 && !descs) return -3;
    if (opts && (!(opts->tol >= 0.0) || opts->max_iter < 0)) return -4;
    if (!out) return -5;
    *out = nullptr;
    for (int64_t i = 0; i < count; ++i) {
        const bfx_solve_desc &d = descs[i];
        if (d.n < 1 || d.n > SMAXN || !d.A || d.lda < d.n || !d.b || !d.x) {
            set_error("bfx_lu_ir_batched_plan_create: descriptor invalid (1 <= n <= 1024, lda >= n, "
                      "non-NULL A, b, x)");
            return (int)(-(100 + (i < 1000000 ? i : 1000000)));
        }
    }
    bfx_solve_plan *p = new bfx_solve_plan();
    p->variant = variant;
    p->count = count;
    if (opts) p->opts = *opts;
    p->h_desc.assign(descs, descs + count);
    // longest first
    std::vector<int64_t> order(count);
    for (int64_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return descs[a].n > descs[b].n; });
    int64_t lu_total = 0, piv_total = 0;
    p->lu_off.resize(count);
    p->piv_off.resize(count);
    for (int64_t i = 0; i < count; ++i) {
        p->lu_off[i] = lu_total;
        p->piv_off[i] = piv_total;
        lu_total += ((descs[i].n * descs[i].n + 63) / 64) * 64;   // 256-byte aligned factors
        piv_total += descs[i].n;
    }
    hipError_t e;
    auto fail = [&](hipError_t err, const char *what) {
        const int rc = hip_fail(err, what);
        solve_plan_free(p);
        return rc;
    };
    const int64_t cn = count > 0 ? count : 1;
    if ((e = hipMalloc(&p->d_lu, sizeof(float) * (lu_total > 0 ? lu_total : 1))) != hipSuccess)
        return fail(e, "hipMalloc(plan factors)");
    if ((e = hipMalloc(&p->d_ipiv, sizeof(int32_t) * (piv_total > 0 ? piv_total : 1))) != hipSuccess)
        return fail(e, "hipMalloc(plan ipiv)");
    if ((e = hipMalloc(&p->d_res, sizeof(bfx_ir_result) * cn)) != hipSuccess)
        return fail(e, "hipMalloc(plan results)");
    if ((e = hipMalloc(&p->d_info, sizeof(int32_t) * cn)) != hipSuccess) return fail(e, "hipMalloc(plan info)");
    if ((e = hipMalloc(&p->d_counter, 256)) != hipSuccess) return fail(e, "hipMalloc(plan counter)");
    if ((e = hipMalloc(&p->d_items, sizeof(SolveItem) * cn)) != hipSuccess) return fail(e, "hipMalloc(plan items)");
    std::vector<SolveItem> items(count);
    for (int64_t k = 0; k < count; ++k) {
        const int64_t i = order[k];
        const bfx_solve_desc &d = descs[i];
        items[k] = SolveItem{d.n, d.A, d.lda, d.b, d.x, p->d_lu + p->lu_off[i], p->d_ipiv + p->piv_off[i],
                             p->d_res + i, p->d_info + i};
    }
    if (count > 0 &&
        (e = hipMemcpy(p->d_items, items.data(), sizeof(SolveItem) * count, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy(plan items)");
    // per-problem baseline workspace
    size_t ws = 0;
    for (int64_t i = 0; i < count; ++i) {
        ws = std::max(ws, bfx_lu_ws_size(descs[i].n));
        ws = std::max(ws, bfx_ir_ws_size(descs[i].n));
    }
    p->ws_bytes = ws;
    if (ws && (e = hipMalloc(&p->d_ws, ws)) != hipSuccess) return fail(e, "hipMalloc(plan workspace)");
    switch (variant) {
        case 1: p->kernel = solve_kernel_for<1>(); break;
        case 3: p->kernel = solve_kernel_for<3>(); break;
        case 6: p->kernel = solve_kernel_for<6>(); break;
        default: p->kernel = solve_kernel_for<9>(); break;
    }
    if ((e = hipFuncSetAttribute(p->kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SOLVE_LDS)) !=
        hipSuccess)
        return fail(e, "hipFuncSetAttribute(solve)");
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return fail(e, "hipDeviceGetAttribute");
    p->grid = (int)std::min<int64_t>(cus, cn);
    if ((e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) != hipSuccess)
        return fail(e, "hipStreamCreate(solve plan)");
    *out = p;
    return BFX_OK;
}

extern "C" int bfx_solve_plan_launch(bfx_solve_plan *p, void *stream) {
    using namespace bfx;
    if (!p) return -1;
    if (p->count == 0) return BFX_OK;
    if (!p->exec) {
        BFX_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(solve_zero_counter, dim3(1), dim3(64), 0, p->cap, p->d_counter);
        double tol = p->opts.tol;
        int max_iter = p->opts.max_iter;
        void *args[] = {&p->d_items, &p->count, &p->d_counter, &tol, &max_iter};
        hipError_t el = hipLaunchKernel(p->kernel, dim3(p->grid), dim3(256), args, SOLVE_LDS, p->cap);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(p->cap, &g);
        if (el != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(el, "persistent solve kernel capture");
        }
        if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
        p->graph = g;
        BFX_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    BFX_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return BFX_OK;
}

extern "C" int bfx_solve_plan_launch_per_problem(bfx_solve_plan *p, void *stream) {
    using namespace bfx;
    if (!p) return -1;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t i = 0; i < p->count; ++i) {
        const bfx_solve_desc &d = p->h_desc[i];
        float *lu = p->d_lu + p->lu_off[i];
        BFX_HIP(hipMemcpy2DAsync(lu, d.n * sizeof(float), d.A, d.lda * sizeof(float), d.n * sizeof(float),
                                 d.n, hipMemcpyDeviceToDevice, s));
        int rc = bfx_lu_factor(p->variant, d.n, lu, d.n, p->d_ipiv + p->piv_off[i], p->d_info + i, p->d_ws,
                               p->ws_bytes, s);
        if (rc) return rc;
        rc = bfx_ir_solve(d.n, d.A, d.lda, lu, d.n, p->d_ipiv + p->piv_off[i], d.b, d.x, &p->opts,
                          p->d_res + i, p->d_ws, p->ws_bytes, s);
        if (rc) return rc;
    }
    return BFX_OK;
}

extern "C" int bfx_solve_plan_results(const bfx_solve_plan *p, bfx_ir_result *results, int32_t *info) {
    using namespace bfx;
    if (!p) return -1;
    BFX_HIP(hipDeviceSynchronize());
    if (results && p->count)
        BFX_HIP(hipMemcpy(results, p->d_res, sizeof(bfx_ir_result) * p->count, hipMemcpyDeviceToHost));
    if (info && p->count)
        BFX_HIP(hipMemcpy(info, p->d_info, sizeof(int32_t) * p->count, hipMemcpyDeviceToHost));
    return BFX_OK;
}

extern "C" int bfx_solve_plan_destroy(bfx_solve_plan *p) {
    if (!p) return -1;
    bfx::solve_plan_free(p);
    return BFX_OK;
}
