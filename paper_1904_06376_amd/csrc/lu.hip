// Blocked right-looking LU with partial pivoting (SGETRF semantics; the
// paper's split-BF16 LU, Sec. I and Sec. IV-A).  For every panel of up to 128
// columns:
//   1. panel_kernel  - FP32 factorisation of the (n-j) x jb panel.  The panel
//      rows are spread over G co-resident workgroups, 256 rows each, held in
//      LDS for the whole panel.  Per column: each workgroup finds its local
//      arg-max (wave shuffles + LDS), publishes the candidate row, one grid
//      barrier, then every workgroup picks the same pivot (largest magnitude,
//      lowest row on ties, as ISAMAX), swaps, divides and applies the rank-1
//      update to its own rows.  One grid barrier per column.
//   2. laswp_kernel  - the panel's row interchanges applied to the columns
//      left and right of the panel.
//   3. trsm_kernel   - U12 = L11^{-1} A12 (unit lower, FP32 FMA chains in
//      index order, one thread per column, L11 in LDS).
//   4. A22 -= L21 x U12 with the split-BF16 GEMM (alpha = -1, beta = 1).
#include <climits>

#include "common.hpp"

namespace bfx {

namespace {
constexpr int PNB = 128;     // panel width
constexpr int PROWS = 256;   // panel rows per workgroup (= threads)
constexpr int MAX_G = 256;   // co-resident workgroups the panel may use
constexpr unsigned SPIN_LIMIT = 1u << 20;  // ~1 s of polling

struct LuWs {
    float *slot_val;    // [2][MAX_G]
    int32_t *slot_idx;  // [2][MAX_G]
    float *slot_row;    // [2][MAX_G][PNB]
    float *diag_row;    // [2][PNB]
    uint32_t *counter;  // grid barrier arrivals
};

size_t lu_ws_layout(LuWs *w, void *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_val = take(sizeof(float) * 2 * MAX_G);
    const size_t o_idx = take(sizeof(int32_t) * 2 * MAX_G);
    const size_t o_row = take(sizeof(float) * 2 * MAX_G * PNB);
    const size_t o_diag = take(sizeof(float) * 2 * PNB);
    const size_t o_cnt = take(sizeof(uint32_t) * 4);
    if (w && base) {
        char *b = (char *)base;
        w->slot_val = (float *)(b + o_val);
        w->slot_idx = (int32_t *)(b + o_idx);
        w->slot_row = (float *)(b + o_row);
        w->diag_row = (float *)(b + o_diag);
        w->counter = (uint32_t *)(b + o_cnt);
    }
    return off;
}

struct PanelArgs {
    float *A;
    int64_t lda, n, j, m;  // m = n - j panel rows
    int w;                 // panel width <= PNB
    int G;                 // workgroups
    int32_t *ipiv, *info;
    LuWs ws;
};
}  // namespace

__device__ __forceinline__ void better(float &v, int &i, float v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// Grid-wide barrier over the G workgroups of the panel: arrivals counted on a
// monotonic counter; every wait is bounded.  On expiry info is set to -1 and
// from then on no barrier of this launch waits, so every wave still exits
// promptly (the factorisation is then reported invalid through info).
__device__ void grid_barrier(uint32_t *counter, uint32_t target, int32_t *info) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1) break;
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    __threadfence();
}

__global__ void __launch_bounds__(PROWS) panel_kernel(PanelArgs a) {
    extern __shared__ float P[];  // [PROWS][w + 1]
    __shared__ float U[PNB], D[PNB];
    __shared__ float red_v[PROWS / 64];
    __shared__ int red_i[PROWS / 64];
    __shared__ int s_piv;

    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w = a.w, ld = w + 1;
    const int64_t row0 = (int64_t)g * PROWS;      // first panel row of this workgroup
    const int64_t pr = row0 + t;                   // panel row owned by this thread
    const bool own = pr < a.m;
    float *Ag = a.A + a.j * a.lda + a.j;           // panel origin

    for (int e = t; e < PROWS * w; e += PROWS) {
        const int r = e / w, q = e % w;
        P[r * ld + q] = (row0 + r < a.m) ? Ag[(row0 + r) * a.lda + q] : 0.0f;
    }
    __syncthreads();

    for (int c = 0; c < w; ++c) {
        const int par = c & 1;
        // ---- local arg-max of |P[., c]| over rows >= c
        float v = (own && pr >= c) ? fabsf(P[t * ld + c]) : -1.0f;
        int idx = own ? (int)pr : INT_MAX;
        if (!(v == v)) v = INFINITY;  // NaN pivots win (and poison the result)
        for (int off = 32; off > 0; off >>= 1) {
            const float v2 = __shfl_xor(v, off);
            const int i2 = __shfl_xor(idx, off);
            better(v, idx, v2, i2);
        }
        if (lane == 0) { red_v[wave] = v; red_i[wave] = idx; }
        __syncthreads();
        if (t == 0) {
            float bv = red_v[0];
            int bi = red_i[0];
            for (int k = 1; k < PROWS / 64; ++k) better(bv, bi, red_v[k], red_i[k]);
            a.ws.slot_val[par * MAX_G + g] = bv;
            a.ws.slot_idx[par * MAX_G + g] = (bv >= 0.0f) ? bi : INT_MAX;
            s_piv = (bv >= 0.0f) ? bi : -1;
        }
        __syncthreads();
        if (s_piv >= 0 && t < w)
            a.ws.slot_row[(par * MAX_G + g) * PNB + t] = P[(s_piv - row0) * ld + t];
        if (c >= row0 && c < row0 + PROWS && t < w)
            a.ws.diag_row[par * PNB + t] = P[(c - row0) * ld + t];
        grid_barrier(a.ws.counter, (uint32_t)(c + 1) * (uint32_t)a.G, a.info);

        // ---- global pivot: every workgroup reduces the same candidates
        if (wave == 0) {
            float bv = -1.0f;
            int bi = INT_MAX, bg = 0;
            for (int k = lane; k < a.G; k += 64) {
                const float v2 = a.ws.slot_val[par * MAX_G + k];
                const int i2 = a.ws.slot_idx[par * MAX_G + k];
                if (v2 > bv || (v2 == bv && i2 < bi)) { bv = v2; bi = i2; bg = k; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const float v2 = __shfl_xor(bv, off);
                const int i2 = __shfl_xor(bi, off);
                const int g2 = __shfl_xor(bg, off);
                if (v2 > bv || (v2 == bv && i2 < bi)) { bv = v2; bi = i2; bg = g2; }
            }
            if (lane == 0) { s_piv = bi; red_i[0] = bg; }
        }
        __syncthreads();
        const int p = s_piv;
        const int pg = red_i[0];
        if (t < w) {
            U[t] = a.ws.slot_row[(par * MAX_G + pg) * PNB + t];
            D[t] = a.ws.diag_row[par * PNB + t];
        }
        __syncthreads();
        const float piv = U[c];
        if (g == 0 && t == 0) {
            a.ipiv[a.j + c] = (int32_t)(a.j + p);
            if (piv == 0.0f && *a.info == 0) *a.info = (int32_t)(a.j + c + 1);  // -1 (expired wait) is kept
        }
        // ---- swap rows c and p, divide, rank-1 update of the own row
        if (own) {
            float *row = P + t * ld;
            if (pr == p && p != c)
                for (int q = 0; q < w; ++q) row[q] = D[q];
            if (pr == c)
                for (int q = 0; q < w; ++q) row[q] = U[q];
            if (pr > c) {
                float l = row[c];
                if (piv != 0.0f) l = l / piv;
                row[c] = l;
                for (int q = c + 1; q < w; ++q) row[q] = fmaf(-l, U[q], row[q]);
            }
        }
        __syncthreads();
    }

    for (int e = t; e < PROWS * w; e += PROWS) {
        const int r = e / w, q = e % w;
        if (row0 + r < a.m) Ag[(row0 + r) * a.lda + q] = P[r * ld + q];
    }
}

__global__ void __launch_bounds__(64) zero_u32(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Row interchanges of rows j..j+w-1 (ipiv) on every column outside the panel.
__global__ void __launch_bounds__(256)
laswp_kernel(float *A, int64_t lda, int64_t n, int64_t j, int w, const int32_t *ipiv) {
    int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (col >= j) col += w;
    if (col >= n) return;
    for (int i = 0; i < w; ++i) {
        const int64_t r = j + i, p = ipiv[r];
        if (p != r) {
            const float x = A[r * lda + col];
            A[r * lda + col] = A[p * lda + col];
            A[p * lda + col] = x;
        }
    }
}

// U12 = L11^{-1} A12.  Each 128-thread workgroup copies 128 columns of A12
// and L11 into LDS; each thread then solves its own column by forward
// substitution in row order, s = a_r - sum_{p<r} L_rp x_p as one FMA chain in
// increasing p (the unblocked algorithm's order), and the block is copied back.
constexpr int TRSM_COLS = 128;
__global__ void __launch_bounds__(TRSM_COLS)
trsm_kernel(float *A, int64_t lda, int64_t n, int64_t j, int w) {
    extern __shared__ float sm[];
    float *L = sm;                    // [PNB][PNB]
    float *X = sm + PNB * PNB;        // [PNB][TRSM_COLS + 1]
    constexpr int XLD = TRSM_COLS + 1;
    const int t = threadIdx.x;
    const int64_t c0 = j + w + (int64_t)blockIdx.x * TRSM_COLS;
    const int ncols = (int)((n - c0 < TRSM_COLS) ? n - c0 : TRSM_COLS);
    for (int e = t; e < PNB * PNB; e += TRSM_COLS) {
        const int i = e / PNB, p = e % PNB;
        L[e] = (i < w && p < i) ? A[(j + i) * lda + j + p] : 0.0f;
    }
    for (int i = 0; i < w; ++i)
        if (t < ncols) X[i * XLD + t] = A[(j + i) * lda + c0 + t];
    __syncthreads();
    if (t < ncols) {
        for (int i = 1; i < w; ++i) {
            float s = X[i * XLD + t];
            const float *li = L + i * PNB;
            for (int p = 0; p < i; ++p) s = fmaf(-li[p], X[p * XLD + t], s);
            X[i * XLD + t] = s;
        }
    }
    __syncthreads();
    for (int i = 1; i < w; ++i)
        if (t < ncols) A[(j + i) * lda + c0 + t] = X[i * XLD + t];
}

static int lu_factor_impl(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv,
                          int32_t *info, void *ws, hipStream_t s) {
    LuWs w;
    lu_ws_layout(&w, ws);
    static bool attr = false;
    if (!attr) {
        BFX_HIP(hipFuncSetAttribute((const void *)panel_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    PROWS * (PNB + 1) * (int)sizeof(float)));
        BFX_HIP(hipFuncSetAttribute((const void *)trsm_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (PNB * PNB + PNB * (TRSM_COLS + 1)) * (int)sizeof(float)));
        attr = true;
    }
    BFX_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), s));
    for (int64_t j = 0; j < n; j += PNB) {
        const int jb = (int)((n - j < PNB) ? n - j : PNB);
        PanelArgs pa;
        pa.A = A; pa.lda = lda; pa.n = n; pa.j = j; pa.m = n - j; pa.w = jb;
        pa.G = (int)ceil_div(n - j, PROWS);
        pa.ipiv = ipiv; pa.info = info; pa.ws = w;
        hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, w.counter, 4);
        BFX_LAUNCH_CHECK("zero_u32");
        void *args[] = {&pa};
        const size_t lds = (size_t)PROWS * (jb + 1) * sizeof(float);
        BFX_HIP(hipLaunchCooperativeKernel((const void *)panel_kernel, dim3(pa.G), dim3(PROWS),
                                           args, (unsigned)lds, s));
        const int64_t others = n - jb;
        if (others > 0) {
            hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)ceil_div(others, 256)), dim3(256), 0, s,
                               A, lda, n, j, jb, ipiv);
            BFX_LAUNCH_CHECK("laswp_kernel");
        }
        const int64_t rest = n - j - jb;
        if (rest <= 0) continue;
        hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)ceil_div(rest, TRSM_COLS)), dim3(TRSM_COLS),
                           (PNB * PNB + PNB * (TRSM_COLS + 1)) * sizeof(float), s, A, lda, n, j, jb);
        BFX_LAUNCH_CHECK("trsm_kernel");
        float *A21 = A + (j + jb) * lda + j;
        float *A12 = A + j * lda + (j + jb);
        float *A22 = A + (j + jb) * lda + (j + jb);
        const int rc = gemm_launch(variant, rest, rest, jb, -1.0f, A21, lda, A12, lda, 1.0f,
                                   A22, lda, nullptr, 0, s);
        if (rc != BFX_OK) return rc;
    }
    return BFX_OK;
}

}  // namespace bfx

extern "C" size_t bfx_lu_ws_size(int64_t n) {
    (void)n;
    return bfx::lu_ws_layout(nullptr, nullptr);
}

extern "C" int bfx_lu_factor(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv,
                             int32_t *info, void *ws, size_t ws_bytes, void *stream) {
    if (variant != 1 && variant != 3 && variant != 6 && variant != 9) return -1;
    if (n < 0) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && !ipiv) return -5;
    if (!info) return -6;
    if (!ws || ws_bytes < bfx_lu_ws_size(n)) return -8;
    if (bfx::ceil_div(n, bfx::PROWS) > bfx::MAX_G) {
        bfx::set_error("bfx_lu_factor: n exceeds 65536 (panel rows must fit in LDS of co-resident workgroups)");
        return -2;
    }
    if (n == 0) {
        BFX_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), (hipStream_t)stream));
        return BFX_OK;
    }
    return bfx::lu_factor_impl(variant, n, A, lda, ipiv, info, ws, (hipStream_t)stream);
}
