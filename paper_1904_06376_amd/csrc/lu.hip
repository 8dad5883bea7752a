// Blocked right-looking LU with partial pivoting (SGETRF semantics; the
// paper's split-BF16 LU, Sec. I and Sec. IV-A).  For every panel of up to 128
// columns:
//   1. panel_kernel  - FP32 factorisation of the (n-j) x jb panel.  The panel
//      rows are spread over G co-resident workgroups, 512 rows each, one row
//      per thread held in registers for the whole panel.  Per column: each
//      workgroup finds its local arg-max (wave shuffles + LDS) and
//      publishes the candidate row and a
//      64-bit header {column tag, |candidate|}; every workgroup then polls the
//      G headers of that column, picks the same pivot (largest magnitude,
//      lowest row on ties, as ISAMAX: workgroups own increasing row ranges),
//      reads the winning row, swaps, divides and applies the rank-1 update to
//      its own rows.  The header exchange is the only grid-wide
//      synchronisation: one round of polling per column, no barrier counter.
//   2. laswp_kernel  - the panel's row interchanges applied to the columns
//      left and right of the panel (composed into one row permutation, each
//      affected row moved once).
//   3. trsm_kernel   - U12 = L11^{-1} A12 (unit lower, FP32 FMA chains in
//      index order; column-oriented steps over register-resident rows).
//   4. A22 -= L21 x U12 with the split-BF16 GEMM (alpha = -1, beta = 1).
#include <climits>

#include "common.hpp"

namespace bfx {

namespace {
constexpr int PNB = 128;     // panel width
constexpr int PROWS = 512;   // panel rows per workgroup (= threads, one row each in registers)
constexpr int MAX_G = 256;   // co-resident workgroups the panel may use
constexpr unsigned SPIN_LIMIT = 1u << 20;  // ~1 s of polling

struct LuWs {
    uint64_t *hdr;      // [2][MAX_G] {tag << 32 | bits(|candidate|)}
    int32_t *slot_idx;  // [2][MAX_G] candidate row (panel-relative)
    float *slot_row;    // [2][MAX_G][PNB] candidate row values
    float *diag_row;    // [2][PNB] row c before the interchange
};

size_t lu_ws_layout(LuWs *w, void *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_hdr = take(sizeof(uint64_t) * 2 * MAX_G);
    const size_t o_idx = take(sizeof(int32_t) * 2 * MAX_G);
    const size_t o_row = take(sizeof(float) * 2 * MAX_G * PNB);
    const size_t o_diag = take(sizeof(float) * 2 * PNB);
    if (w && base) {
        char *b = (char *)base;
        w->hdr = (uint64_t *)(b + o_hdr);
        w->slot_idx = (int32_t *)(b + o_idx);
        w->slot_row = (float *)(b + o_row);
        w->diag_row = (float *)(b + o_diag);
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

// Each thread holds one panel row in registers, r[0..PNB-1], in a layout
// that keeps the current column in r[0]: after k eliminations (k = the
// column index for rows still below the diagonal) r[0 .. w-k-1] hold columns
// k .. w-1, r[PNB-k .. PNB-1] hold the multipliers l_0 .. l_{k-1}, and the
// registers between are padding.  An elimination shifts the row left by one
// (r[i] = r[i+1] - l U[i+1] on the live part, a plain shift elsewhere) and
// puts the new multiplier in r[PNB-1]; all register indices are static.  Rows
// that reach the diagonal freeze.  Two rows that swap at column c were both
// shifted c times, so their register images are exchanged as they are.
__global__ void __launch_bounds__(PROWS, 1) panel_kernel(PanelArgs a) {
    __shared__ __align__(16) float U[PNB], D[PNB], rowbuf[PNB], diagbuf[PNB];
    __shared__ float red_v[PROWS / 64];
    __shared__ int red_i[PROWS / 64];
    __shared__ int s_piv, s_win;
    __shared__ float s_val;

    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w = a.w;
    const int64_t row0 = (int64_t)g * PROWS;      // first panel row of this workgroup
    const int64_t pr = row0 + t;                   // panel row owned by this thread
    const bool own = pr < a.m;
    float *Ag = a.A + a.j * a.lda + a.j;           // panel origin
    float r[PNB];
#pragma unroll
    for (int k = 0; k < PNB; ++k) r[k] = (own && k < w) ? Ag[pr * a.lda + k] : 0.0f;

    for (int c = 0; c < w; ++c) {
        const int par = c & 1;
        const uint32_t tag = (uint32_t)(a.j + c + 1);   // never 0 (headers start zeroed)
        const bool active = own && pr >= c;             // rows at or below the diagonal
        // ---- local arg-max of |column c| over rows >= c
        float v = active ? fabsf(r[0]) : -1.0f;
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
            s_val = bv;
            s_piv = (bv >= 0.0f) ? bi : -1;
        }
        __syncthreads();
        // ---- the candidate row and row c (register images) to LDS
        if (own && pr == s_piv) {
#pragma unroll
            for (int k = 0; k < PNB; ++k) rowbuf[k] = r[k];
        }
        if (own && pr == c) {
#pragma unroll
            for (int k = 0; k < PNB; ++k) diagbuf[k] = r[k];
        }
        __syncthreads();
        // ---- wave 0 publishes them, then the header with release order
        // (covering the wave's own stores)
        if (wave == 0) {
            const bool has_c = c >= row0 && c < row0 + PROWS;
            for (int q = lane; q < PNB; q += 64) {
                if (s_piv >= 0) a.ws.slot_row[(par * MAX_G + g) * PNB + q] = rowbuf[q];
                if (has_c) a.ws.diag_row[par * PNB + q] = diagbuf[q];
            }
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                a.ws.slot_idx[par * MAX_G + g] = s_piv;
                const uint64_t h = ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(s_val);
                __hip_atomic_store(&a.ws.hdr[par * MAX_G + g], h, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // ---- every wave polls 64 of the G headers (bounded wait), then the
        // largest candidate wins, the lowest workgroup on ties
        {
            const int k = wave * 64 + lane;
            float bv = -2.0f;
            int bg = INT_MAX;
            if (k < a.G) {
                uint64_t h = 0;
                unsigned spins = 0;
                for (;;) {
                    h = __hip_atomic_load(&a.ws.hdr[par * MAX_G + k], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    if ((uint32_t)(h >> 32) == tag) {
                        // acquire: the candidate rows published before it are visible
                        (void)__hip_atomic_load(&a.ws.hdr[par * MAX_G + k], __ATOMIC_ACQUIRE,
                                                __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    if (__hip_atomic_load(a.info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1) break;
                    if (++spins > SPIN_LIMIT) {
                        __hip_atomic_store(a.info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                bv = __uint_as_float((uint32_t)h);
                bg = k;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const float v2 = __shfl_xor(bv, off);
                const int g2 = __shfl_xor(bg, off);
                better(bv, bg, v2, g2);
            }
            if (lane == 0) { red_v[wave] = bv; red_i[wave] = bg; }
        }
        __syncthreads();
        if (t == 0) {
            float bv = red_v[0];
            int bg = red_i[0];
            for (int k = 1; k < PROWS / 64; ++k) better(bv, bg, red_v[k], red_i[k]);
            // a wait that expired leaves bg possibly without a published row:
            // fall back to this workgroup's own slot (the result is invalid
            // anyway and reported through info = -1)
            s_win = (bg < a.G) ? bg : g;
        }
        __syncthreads();
        const int pg = s_win;
        if (t < PNB) {
            U[t] = a.ws.slot_row[(par * MAX_G + pg) * PNB + t];
            D[t] = a.ws.diag_row[par * PNB + t];
        }
        if (t == 0) s_piv = a.ws.slot_idx[par * MAX_G + pg];
        __syncthreads();
        // a valid pivot row is >= c; anything else only follows an expired wait
        const int p = (s_piv >= c && s_piv < a.m) ? s_piv : c;
        const float piv = U[0];
        if (g == 0 && t == 0) {
            a.ipiv[a.j + c] = (int32_t)(a.j + p);
            if (piv == 0.0f && *a.info == 0) *a.info = (int32_t)(a.j + c + 1);  // -1 (expired wait) is kept
        }
        // ---- swap rows c and p, divide, shift-update the rows below
        if (active) {
            if (pr == p && p != c) {
#pragma unroll
                for (int k = 0; k < PNB; ++k) r[k] = D[k];
            }
            if (pr == c) {
#pragma unroll
                for (int k = 0; k < PNB; ++k) r[k] = U[k];
            } else {
                float l = r[0];
                if (piv != 0.0f) l = l / piv;
                const int live = w - c;   // r[0 .. live-1] are columns c .. w-1
                // blocks of 8 registers: all updated, all shifted, or mixed
#pragma unroll
                for (int b = 0; b < PNB / 8; ++b) {
                    if (8 * b + 8 <= live - 1) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int k = 8 * b + i;
                            if (k < PNB - 1) r[k] = fmaf(-l, U[k + 1], r[k + 1]);
                        }
                    } else if (8 * b >= live - 1) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int k = 8 * b + i;
                            if (k < PNB - 1) r[k] = r[k + 1];
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int k = 8 * b + i;
                            if (k < PNB - 1) r[k] = (k < live - 1) ? fmaf(-l, U[k + 1], r[k + 1]) : r[k + 1];
                        }
                    }
                }
                r[PNB - 1] = l;
            }
        }
    }

    // ---- write back: register k of a row shifted s times holds column s + k
    // (k < w - s) or multiplier k - (PNB - s) (k >= PNB - s)
    if (own) {
        const int sh = (pr < w) ? (int)pr : w;
#pragma unroll
        for (int k = 0; k < PNB; ++k) {
            int col = -1;
            if (k < w - sh) col = sh + k;
            else if (k >= PNB - sh) col = k - (PNB - sh);
            if (col >= 0) Ag[pr * a.lda + col] = r[k];
        }
    }
}

__global__ void __launch_bounds__(256) zero_u64(uint64_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += 256) p[i] = 0ull;
}

// Row interchanges of rows j..j+w-1 (ipiv, applied in order, LAPACK laswp
// semantics) on every column outside the panel.
constexpr int SWP_COLS = 64;       // columns per workgroup
constexpr int SWP_THREADS = 256;   // 4 waves: wave v moves affected rows v, v+4, ...
constexpr int SWP_MAXR = 2 * PNB;  // affected rows: the panel rows and at most w others
// The w interchanges compose into one permutation of at most 2w rows: the
// affected positions are the panel rows 0..w-1 and every pivot row beyond
// them.  Position p receives the old row sigma(p), sigma = tau_0 o tau_1 o
// ... o tau_{w-1} (tau_i swaps i and ipiv[i]); each thread evaluates sigma
// for its positions by applying the transpositions in reverse order.  Then
// every affected row of the workgroup's 64 columns is loaded (coalesced
// 256-byte row segments, many loads in flight), all loads complete before
// the barrier, and the rows are stored at their new positions.
__global__ void __launch_bounds__(SWP_THREADS)
laswp_kernel(float *A, int64_t lda, int64_t n, int64_t j, int w, const int32_t *ipiv) {
    __shared__ int sp[PNB], dpos[SWP_MAXR], spos[SWP_MAXR];
    __shared__ int s_nd;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int i = t; i < w; i += SWP_THREADS) {
        const int64_t q = ipiv[j + i] - j;  // >= i for a valid factorisation
        sp[i] = (q >= i && q < n - j) ? (int)q : i;
    }
    if (t == 0) s_nd = w;
    __syncthreads();
    if (t < w) {
        dpos[t] = t;
        const int q = sp[t];
        bool first = q >= w;
        for (int k = 0; k < t && first; ++k) first = sp[k] != q;
        if (first) dpos[atomicAdd(&s_nd, 1)] = q;
    }
    __syncthreads();
    const int nd = s_nd;
    for (int e = t; e < nd; e += SWP_THREADS) {
        int pos = dpos[e];
        for (int i = w - 1; i >= 0; --i) {
            const int q = sp[i];
            pos = (pos == i) ? q : ((pos == q) ? i : pos);
        }
        spos[e] = pos;
    }
    __syncthreads();
    int64_t col = (int64_t)blockIdx.x * SWP_COLS + lane;
    if (col >= j) col += w;
    const bool ok = col < n;
    constexpr int PER = SWP_MAXR / 4;   // rows per wave
    float v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = wv + 4 * k;
        v[k] = (ok && e < nd) ? A[(j + spos[e]) * lda + col] : 0.0f;
    }
    // every load of the workgroup has returned before any row is overwritten
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = wv + 4 * k;
        if (ok && e < nd) A[(j + dpos[e]) * lda + col] = v[k];
    }
}

// U12 = L11^{-1} A12 (unit lower L11, jb x jb).  Column-oriented forward
// substitution: at step p the now final row p of X is broadcast and every row
// i > p is updated, x_i = fma(-L_ip, x_p, x_i) -- for each element the same
// FMA chain, in increasing p, as the row-oriented algorithm.  A 256-thread
// workgroup owns 64 columns; wave h keeps rows 32h .. 32h+31 of its column in
// registers, L11 is staged transposed in LDS (rows padded to 132 floats).
// Steps are unrolled in blocks of 32 so that register indices are static.
constexpr int TRSM_COLS = 64;
constexpr int TRSM_LD = PNB + 4;
constexpr size_t TRSM_LDS = (size_t)PNB * TRSM_LD * sizeof(float);
__global__ void __launch_bounds__(256, 2)
trsm_kernel(float *A, int64_t lda, int64_t n, int64_t j, int w) {
    extern __shared__ __align__(16) float Lt[];   // Lt[p * TRSM_LD + i] = L11[i][p]
    __shared__ float xb[TRSM_COLS];
    const int t = threadIdx.x, c = t & 63, h = t >> 6;
    const int64_t col = j + w + (int64_t)blockIdx.x * TRSM_COLS + c;
    const bool ok = col < n;
    for (int e = t; e < PNB * PNB; e += 256) {
        const int i = e / PNB, p = e % PNB;
        Lt[p * TRSM_LD + i] = (i < w && p < i) ? A[(j + i) * lda + j + p] : 0.0f;
    }
    float x[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const int i = 32 * h + k;
        x[k] = (ok && i < w) ? A[(j + i) * lda + col] : 0.0f;
    }
    __syncthreads();
    for (int hp = 0; hp < 4; ++hp) {
        if (32 * hp >= w - 1) break;   // uniform
#pragma unroll
        for (int kp = 0; kp < 32; ++kp) {
            const int p = 32 * hp + kp;
            if (h == hp) xb[c] = x[kp];
            __syncthreads();
            const float xp = xb[c];
            const float *lp = Lt + p * TRSM_LD + 32 * h;   // L11[32h + k][p]
            if (h > hp) {
#pragma unroll
                for (int k = 0; k < 32; ++k) x[k] = fmaf(-lp[k], xp, x[k]);
            } else if (h == hp) {
#pragma unroll
                for (int k = kp + 1; k < 32; ++k) x[k] = fmaf(-lp[k], xp, x[k]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        const int i = 32 * h + k;
        if (ok && i >= 1 && i < w) A[(j + i) * lda + col] = x[k];
    }
}

static int lu_factor_impl(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv,
                          int32_t *info, void *ws, hipStream_t s) {
    LuWs w;
    lu_ws_layout(&w, ws);
    static bool attr = false;
    if (!attr) {
        BFX_HIP(hipFuncSetAttribute((const void *)trsm_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)TRSM_LDS));
        attr = true;
    }
    BFX_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(256), 0, s, w.hdr, 2 * MAX_G);
    BFX_LAUNCH_CHECK("zero_u64");
    for (int64_t j = 0; j < n; j += PNB) {
        const int jb = (int)((n - j < PNB) ? n - j : PNB);
        PanelArgs pa;
        pa.A = A; pa.lda = lda; pa.n = n; pa.j = j; pa.m = n - j; pa.w = jb;
        pa.G = (int)ceil_div(n - j, PROWS);
        pa.ipiv = ipiv; pa.info = info; pa.ws = w;
        void *args[] = {&pa};
        BFX_HIP(hipLaunchCooperativeKernel((const void *)panel_kernel, dim3(pa.G), dim3(PROWS),
                                           args, 0, s));
        const int64_t others = n - jb;
        if (others > 0) {
            hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)ceil_div(others, SWP_COLS)), dim3(SWP_THREADS),
                               0, s, A, lda, n, j, jb, ipiv);
            BFX_LAUNCH_CHECK("laswp_kernel");
        }
        const int64_t rest = n - j - jb;
        if (rest <= 0) continue;
        hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)ceil_div(rest, TRSM_COLS)), dim3(256), TRSM_LDS, s,
                           A, lda, n, j, jb);
        BFX_LAUNCH_CHECK("trsm_kernel");
        float *A21 = A + (j + jb) * lda + j;
        float *A12 = A + j * lda + (j + jb);
        float *A22 = A + (j + jb) * lda + (j + jb);
        // variant 0: the plain FP32 vector GEMM (an SGETRF built on SGEMM, the
        // comparator of Sec. IV-A's LU experiment)
        const int rc = variant == 0
                           ? bfx_sgemm_fp32(rest, rest, jb, -1.0f, A21, lda, A12, lda, 1.0f, A22, lda,
                                            nullptr, 0, (void *)s)
                           : gemm_launch(variant, rest, rest, jb, -1.0f, A21, lda, A12, lda, 1.0f,
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
    if (variant != 0 && variant != 1 && variant != 3 && variant != 6 && variant != 9) return -1;
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
