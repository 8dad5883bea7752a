// Iterative refinement in residual form (Sec. III) and the FP32 LU solve.
//
//   x0 = LUsolve32(b);  repeat: r = b - A x (FP64, A promoted exactly),
//   eta = |r|_inf / (|A|_inf |x|_inf + |b|_inf), stop when eta <= tol;
//   s = |r|_inf, d = s * LUsolve32(r / s), x += d (FP64).
//
// Only the cubic LU is low precision; every quadratic step is FP64 except the
// two FP32 triangular solves with the stored factors.  Kernels:
//   residual_kernel  one workgroup per row, FP64 FMA, |r|_inf by atomicMax on
//                    the bit pattern of a non-negative double (order-free);
//   trsv_kernel      blocked triangular solve without a global barrier: each
//                    workgroup takes the next block row from a ticket counter,
//                    waits (bounded) on the completion flags of the blocks it
//                    depends on, adds their contribution, solves its 128 x 128
//                    diagonal block in one wave and publishes its flag;
//   perm_kernel      the row permutation of ipiv, composed once per solve
//                    (every position evaluated in parallel).
// The host reads |r|_inf and |x|_inf once per step to apply the stopping rule.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace bfx {

namespace {
constexpr int TB = 128;
constexpr size_t TRSV_LDS = sizeof(float) * TB * (TB + 1);
constexpr unsigned SPIN_LIMIT = 1u << 20;  // ~1 s of polling

enum { S_NORMA = 0, S_NORMB = 1, S_RN = 2, S_XN = 3, S_NSCAL = 8 };

struct IrWs {
    int32_t *perm;
    float *w;
    double *r;
    int32_t *flags;   // [nblk]
    uint32_t *ticket; // [4]
    unsigned long long *scal;  // [S_NSCAL]
    int32_t *err;
};

size_t ir_ws_layout(IrWs *w, void *base, int64_t n) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const int64_t nb = ceil_div(n > 0 ? n : 1, TB);
    const size_t o_perm = take(sizeof(int32_t) * (n > 0 ? n : 1));
    const size_t o_w = take(sizeof(float) * (n > 0 ? n : 1));
    const size_t o_r = take(sizeof(double) * (n > 0 ? n : 1));
    const size_t o_f = take(sizeof(int32_t) * nb);
    const size_t o_t = take(sizeof(uint32_t) * 4);
    const size_t o_s = take(sizeof(unsigned long long) * S_NSCAL);
    const size_t o_e = take(sizeof(int32_t) * 4);
    if (w && base) {
        char *b = (char *)base;
        w->perm = (int32_t *)(b + o_perm);
        w->w = (float *)(b + o_w);
        w->r = (double *)(b + o_r);
        w->flags = (int32_t *)(b + o_f);
        w->ticket = (uint32_t *)(b + o_t);
        w->scal = (unsigned long long *)(b + o_s);
        w->err = (int32_t *)(b + o_e);
    }
    return off;
}
}  // namespace

__device__ __forceinline__ void atomic_max_abs(unsigned long long *dst, double v) {
    // |v| as a non-negative double orders like its bit pattern (NaN above Inf)
    atomicMax(dst, (unsigned long long)__double_as_longlong(fabs(v)));
}

__global__ void __launch_bounds__(256) zero_i32(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

// Compose the interchanges ipiv[0..n) into perm: (P v)[i] = v[perm[i]], that
// is perm[i] = tau_0(tau_1(...tau_{n-1}(i))) with tau_k the swap of k and
// ipiv[k] (applying the swaps to v in order k = 0, 1, ... gives exactly that).
// Each thread evaluates the composition for its own position by scanning the
// interchanges backwards (staged in LDS when they fit), so the positions are
// computed in parallel instead of replaying the swaps one after another.
__global__ void __launch_bounds__(256) perm_kernel(const int32_t *ipiv, int64_t n, int32_t *perm,
                                                   int use_lds) {
    extern __shared__ int32_t sp[];
    const int32_t *iv = ipiv;
    if (use_lds) {
        for (int64_t i = threadIdx.x; i < n; i += 256) sp[i] = ipiv[i];
        __syncthreads();
        iv = sp;
    }
    const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pos >= n) return;
    int32_t p = (int32_t)pos;
    for (int32_t i = (int32_t)n - 1; i >= 0; --i) {
        const int32_t q = iv[i];
        p = (p == i) ? q : ((p == q) ? i : p);
    }
    perm[pos] = p;
}

// w[i] = (float)(src[perm[i]] / div)   (src FP64)
__global__ void __launch_bounds__(256)
gather_f64_to_f32(const double *src, const int32_t *perm, double div, float *w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = (float)(src[perm[i]] / div);
}

__global__ void __launch_bounds__(256)
gather_f32(const float *src, const int32_t *perm, float *w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = src[perm[i]];
}

__global__ void __launch_bounds__(256) copy_f32(const float *src, float *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// x = (double) w   (init)   or   x += s * (double) w   (update)
__global__ void __launch_bounds__(256)
update_x(double *x, const float *w, double s, int init, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        x[i] = init ? (double)w[i] : fma(s, (double)w[i], x[i]);
}

template <typename T>
__device__ __forceinline__ T block_sum_256(T v, T *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// r_i = b_i - sum_j A_ij x_j in FP64; |r|_inf into scal[S_RN].
__global__ void __launch_bounds__(256)
residual_kernel(const float *A, int64_t lda, int64_t n, const double *b, const double *x,
                double *r, unsigned long long *scal, int vec) {
    __shared__ double red[4];
    const int64_t row = blockIdx.x;
    const float *a = A + row * lda;
    double s = 0.0;
    if (vec) {
        for (int64_t j = 4 * threadIdx.x; j + 3 < n; j += 1024) {
            const float4 v = *reinterpret_cast<const float4 *>(a + j);
            s = fma((double)v.x, x[j], s);
            s = fma((double)v.y, x[j + 1], s);
            s = fma((double)v.z, x[j + 2], s);
            s = fma((double)v.w, x[j + 3], s);
        }
        for (int64_t j = (n & ~int64_t(3)) + threadIdx.x; j < n; j += 256) s = fma((double)a[j], x[j], s);
    } else {
        for (int64_t j = threadIdx.x; j < n; j += 256) s = fma((double)a[j], x[j], s);
    }
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) {
        const double ri = b[row] - s;
        r[row] = ri;
        atomic_max_abs(scal + S_RN, ri);
    }
}

// |A|_inf = max_i sum_j |A_ij| (FP64) into scal[S_NORMA].
__global__ void __launch_bounds__(256)
mat_norm_kernel(const float *A, int64_t lda, int64_t n, unsigned long long *scal) {
    __shared__ double red[4];
    const float *a = A + (int64_t)blockIdx.x * lda;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) s += fabs((double)a[j]);
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) atomic_max_abs(scal + S_NORMA, s);
}

__global__ void __launch_bounds__(256)
vec_absmax_kernel(const double *v, int64_t n, unsigned long long *dst) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double a = fabs(v[i]);
        if (a > m || a != a) m = a;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off);
        if (o > m || o != o) m = o;
    }
    if ((threadIdx.x & 63) == 0) atomic_max_abs(dst, m);
}

// Value of v in lane l (l uniform), through v_readlane.
__device__ __forceinline__ float bcast_lane(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double bcast_lane(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Blocked triangular solve with the FP32 LU factors, in place on y; T is the
// arithmetic and vector type (float for LU-IR, double for the GMRES
// preconditioner).  lower = 1: unit lower L (forward); lower = 0: upper U
// (backward, divides).  One workgroup per block row of TB = 128 rows, taken in
// dependency order from a ticket counter.  Off-diagonal part: wave w owns rows
// 16w .. 16w+15 of the block row; for every dependency block its 64 lanes
// read 2 consecutive columns each (one coalesced 512-byte load per row) and
// accumulate per row in column order, the 16 row sums being reduced across
// the wave at the end.  The factor values of the next dependency are loaded
// before waiting for it.  Diagonal block: one wave, lane l holding rows l and
// l + 64, substitution in column order with the diagonal block in LDS.
template <typename T>
__global__ void __launch_bounds__(512)
trsv_kernel(const float *LU, int64_t ld, int64_t n, T *y, int32_t *flags, uint32_t *ticket,
            int32_t *err, int lower) {
    extern __shared__ float Ld[];   // [TB][TB + 1] diagonal block
    __shared__ int s_blk;
    __shared__ int64_t s_known;
    __shared__ T rhs[TB];
    constexpr int LDD = TB + 1;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t nblk = ceil_div(n, TB);
    if (t == 0) s_blk = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t blk = lower ? s_blk : nblk - 1 - s_blk;
    const int64_t r0 = blk * TB;
    const int rows = (int)((n - r0 < TB) ? n - r0 : TB);
    // diagonal block to LDS (independent of other blocks)
    for (int e = t; e < TB * TB; e += 512) {
        const int i = e / TB, c = e % TB;
        Ld[i * LDD + c] = (i < rows && c < rows) ? LU[(r0 + i) * ld + r0 + c] : 0.0f;
    }
    const int64_t nb_dep = lower ? blk : nblk - 1 - blk;
    // rows 16 wave .. 16 wave + 15 of this block row (clamped: rows past the
    // end of the matrix re-read the last row and are never stored)
    const float *lrow[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int rr = 16 * wave + q;
        lrow[q] = LU + (r0 + (rr < rows ? rr : rows - 1)) * ld;
    }
    auto col0 = [&](int64_t d) { return (lower ? d : nblk - 1 - d) * TB + 2 * lane; };
    float lc[16][2], ln[16][2];
    auto load = [&](float (&dst)[16][2], int64_t c) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            dst[q][0] = (c < n) ? lrow[q][c] : 0.0f;
            dst[q][1] = (c + 1 < n) ? lrow[q][c + 1] : 0.0f;
        }
    };
    T acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0;
    if (nb_dep > 0) load(lc, col0(0));
    int64_t known = 0;  // dependencies known complete
    for (int64_t d = 0; d < nb_dep; ++d) {
        const int64_t jb = lower ? d : nblk - 1 - d;
        if (d + 1 < nb_dep) load(ln, col0(d + 1));
        if (d >= known) {
            // A block completes only after every block before it in this
            // order, so one acquire of the furthest flag known set covers all
            // earlier blocks; polls are relaxed.
            if (t == 0) {
                unsigned spins = 0;
                while (__hip_atomic_load(flags + jb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                    if (++spins > SPIN_LIMIT) { atomicExch(err, 1); break; }
                    __builtin_amdgcn_s_sleep(1);
                }
                int64_t e = d + 1;
                while (e < nb_dep &&
                       __hip_atomic_load(flags + (lower ? e : nblk - 1 - e), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) != 0)
                    ++e;
                (void)__hip_atomic_load(flags + (lower ? e - 1 : nblk - e), __ATOMIC_ACQUIRE,
                                        __HIP_MEMORY_SCOPE_AGENT);
                s_known = e;
            }
            __syncthreads();
            known = s_known;
        }
        const int64_t c = jb * TB + 2 * lane;
        const T y0 = (c < n) ? y[c] : (T)0, y1 = (c + 1 < n) ? y[c + 1] : (T)0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            acc[q] = fma((T)lc[q][0], y0, acc[q]);
            acc[q] = fma((T)lc[q][1], y1, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) { lc[q][0] = ln[q][0]; lc[q][1] = ln[q][1]; }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    if (lane < 16) {
        // lane q publishes row 16 wave + q (static register index via a select chain)
        T v = acc[0];
#pragma unroll
        for (int q = 1; q < 16; ++q) if (lane == q) v = acc[q];
        const int rr = 16 * wave + lane;
        if (rr < rows) rhs[rr] = y[r0 + rr] - v;
    }
    __syncthreads();
    if (t < 64) {
        // Column c's solution value is read with v_readlane (c is uniform),
        // so it is a wave-uniform operand; every lane computes the FMA and a
        // select keeps it only for the rows it applies to (no exec-mask
        // changes; rows it does not apply to keep their value even when the
        // product is not finite).  The LDS operands of 8 columns
        // are loaded one chunk ahead.  Backward solve on the rows scaled by
        // the reciprocals of their diagonal entries (products rounded once,
        // formed off the dependency chain).
        T v0 = (lane < rows) ? rhs[lane] : (T)0;
        T v1 = (lane + 64 < rows) ? rhs[lane + 64] : (T)0;
        const float *l0 = Ld + lane * LDD, *l1 = Ld + (lane + 64) * LDD;
        float a0[8], a1[8], b0[8], b1[8];
        const int nch = (rows + 7) / 8;
        if (lower) {
            // unit diagonal; columns >= rows of the block hold zeros
#pragma unroll
            for (int k = 0; k < 8; ++k) { a0[k] = l0[k]; a1[k] = l1[k]; }
            for (int ch = 0; ch < nch; ++ch) {
                const int cn = 8 * (ch + 1 < nch ? ch + 1 : ch);
#pragma unroll
                for (int k = 0; k < 8; ++k) { b0[k] = l0[cn + k]; b1[k] = l1[cn + k]; }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int c = 8 * ch + k;
                    const T yc = bcast_lane(c < 64 ? v0 : v1, c & 63);
                    const T u0 = fma(-(T)a0[k], yc, v0), u1 = fma(-(T)a1[k], yc, v1);
                    v0 = (lane > c) ? u0 : v0;
                    v1 = (lane + 64 > c) ? u1 : v1;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) { a0[k] = b0[k]; a1[k] = b1[k]; }
            }
        } else {
            // Rows scaled by the reciprocal of their diagonal entry (each lane
            // holds those of its two rows): U' = D^-1 U has a unit diagonal
            // and the chain per column is one broadcast and one FMA.
            const T rd0 = (lane < rows) ? (T)1 / (T)l0[lane] : (T)0;
            const T rd1 = (lane + 64 < rows) ? (T)1 / (T)l1[lane + 64] : (T)0;
            v0 *= rd0;
            v1 *= rd1;
            const int top = 8 * (nch - 1);
#pragma unroll
            for (int k = 0; k < 8; ++k) { a0[k] = l0[top + k]; a1[k] = l1[top + k]; }
            for (int ch = nch - 1; ch >= 0; --ch) {
                const int cn = 8 * (ch > 0 ? ch - 1 : 0);
#pragma unroll
                for (int k = 0; k < 8; ++k) { b0[k] = l0[cn + k]; b1[k] = l1[cn + k]; }
#pragma unroll
                for (int k = 7; k >= 0; --k) {
                    const int c = 8 * ch + k;
                    if (c < rows) {
                        const T yc = bcast_lane(c < 64 ? v0 : v1, c & 63);
                        const T u0 = fma(-((T)a0[k] * rd0), yc, v0), u1 = fma(-((T)a1[k] * rd1), yc, v1);
                        v0 = (lane < c) ? u0 : v0;
                        v1 = (lane + 64 < c) ? u1 : v1;
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) { a0[k] = b0[k]; a1[k] = b1[k]; }
            }
        }
        if (lane < rows) y[r0 + lane] = v0;
        if (lane + 64 < rows) y[r0 + 64 + lane] = v1;
        __builtin_amdgcn_wave_barrier();
        // the release covers wave 0's stores of y
        if (t == 0) __hip_atomic_store(flags + blk, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}


// ---------------------------------------------------------------------------
// GMRES-IR pieces (all FP64 vectors).
// ---------------------------------------------------------------------------
// y = A x, A promoted exactly, one workgroup per row, fixed-order reduction.
__global__ void __launch_bounds__(256)
matvec_kernel(const float *A, int64_t lda, int64_t n, const double *x, double *y, int vec) {
    __shared__ double red[4];
    const int64_t row = blockIdx.x;
    const float *a = A + row * lda;
    double s = 0.0;
    if (vec) {
        for (int64_t j = 4 * threadIdx.x; j + 3 < n; j += 1024) {
            const float4 v = *reinterpret_cast<const float4 *>(a + j);
            s = fma((double)v.x, x[j], s);
            s = fma((double)v.y, x[j + 1], s);
            s = fma((double)v.z, x[j + 2], s);
            s = fma((double)v.w, x[j + 3], s);
        }
        for (int64_t j = (n & ~int64_t(3)) + threadIdx.x; j < n; j += 256) s = fma((double)a[j], x[j], s);
    } else {
        for (int64_t j = threadIdx.x; j < n; j += 256) s = fma((double)a[j], x[j], s);
    }
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) y[row] = s;
}

__global__ void __launch_bounds__(256)
gather_f64(const double *v, const int32_t *perm, double *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = v[perm[i]];
}

// h[j] = <w, V_j>, j < k: one workgroup per j, fixed-order tree (deterministic).
__global__ void __launch_bounds__(256)
dots_kernel(const double *V, int64_t ldv, const double *w, int64_t n, double *h) {
    __shared__ double red[4];
    const double *v = V + (int64_t)blockIdx.x * ldv;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(v[i], w[i], s);
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) h[blockIdx.x] = s;
}

// w -= sum_{j<k} h_j V_j   (init = 0)   or   x += sum_{j<k} h_j V_j   (sign = +1)
__global__ void __launch_bounds__(256)
combine_kernel(const double *V, int64_t ldv, const double *h, int k, double *w, int64_t n,
               double sign) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double acc = w[i];
        for (int j = 0; j < k; ++j) acc = fma(sign * h[j], V[(int64_t)j * ldv + i], acc);
        w[i] = acc;
    }
}

__global__ void __launch_bounds__(256)
scale_f64(const double *w, double div, double *v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        v[i] = w[i] / div;
}

static unsigned grid_for(int64_t n) {
    int64_t b = ceil_div(n, 256);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// In-place solve of (LU) y = y: T = float on the workspace vector (LU-IR),
// T = double for the GMRES preconditioner.
template <typename T>
static int lu_solve_vec(int64_t n, const float *LU, int64_t ldlu, T *y, const IrWs &w,
                        hipStream_t s) {
    const int64_t nb = ceil_div(n, TB);
    static bool attr = false;
    if (!attr) {
        BFX_HIP(hipFuncSetAttribute((const void *)trsv_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)TRSV_LDS));
        attr = true;
    }
    for (int lower = 1; lower >= 0; --lower) {
        hipLaunchKernelGGL(zero_i32, dim3(grid_for(nb)), dim3(256), 0, s, w.flags, nb);
        hipLaunchKernelGGL(zero_i32, dim3(1), dim3(256), 0, s, (int32_t *)w.ticket, 4);
        hipLaunchKernelGGL(trsv_kernel<T>, dim3((unsigned)nb), dim3(512), TRSV_LDS, s, LU, ldlu, n, y,
                           w.flags, w.ticket, w.err, lower);
        BFX_LAUNCH_CHECK("trsv_kernel");
    }
    return BFX_OK;
}

static int lu_solve_ws(int64_t n, const float *LU, int64_t ldlu, const IrWs &w, hipStream_t s) {
    return lu_solve_vec<float>(n, LU, ldlu, w.w, w, s);
}

static int compose_perm(int64_t n, const int32_t *ipiv, const IrWs &w, hipStream_t s) {
    const size_t lds = sizeof(int32_t) * (size_t)n;
    const int use_lds = lds <= 160 * 1024 - 1024;
    if (use_lds) {
        static size_t attr = 0;
        if (attr < lds) {
            BFX_HIP(hipFuncSetAttribute((const void *)perm_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            attr = lds;
        }
    }
    hipLaunchKernelGGL(perm_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), use_lds ? lds : 0, s, ipiv, n,
                       w.perm, use_lds);
    BFX_LAUNCH_CHECK("perm_kernel");
    return BFX_OK;
}

static int check_err(const IrWs &w, hipStream_t s) {
    int32_t e = 0;
    BFX_HIP(hipMemcpyAsync(&e, w.err, sizeof e, hipMemcpyDeviceToHost, s));
    BFX_HIP(hipStreamSynchronize(s));
    if (e) {
        set_error("triangular solve: a bounded wait on a block flag expired");
        return BFX_E_INTERNAL;
    }
    return BFX_OK;
}

static double bits_to_double(unsigned long long u) {
    double d;
    memcpy(&d, &u, sizeof d);
    return d;
}

}  // namespace bfx

extern "C" size_t bfx_ir_ws_size(int64_t n) {
    return bfx::ir_ws_layout(nullptr, nullptr, n < 0 ? 0 : n);
}

extern "C" int bfx_lu_solve_f32(int64_t n, const float *LU, int64_t ldlu, const int32_t *ipiv,
                                float *rhs, void *ws, size_t ws_bytes, void *stream) {
    if (n < 0) return -1;
    if (n > 0 && !LU) return -2;
    if (ldlu < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !ipiv) return -4;
    if (n > 0 && !rhs) return -5;
    if (!ws || ws_bytes < bfx_ir_ws_size(n)) return -7;
    if (n == 0) return BFX_OK;
    hipStream_t s = (hipStream_t)stream;
    bfx::IrWs w;
    bfx::ir_ws_layout(&w, ws, n);
    hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, w.err, 4);
    int rc = bfx::compose_perm(n, ipiv, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::gather_f32, dim3(bfx::grid_for(n)), dim3(256), 0, s, rhs, w.perm, w.w, n);
    rc = bfx::lu_solve_ws(n, LU, ldlu, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::copy_f32, dim3(bfx::grid_for(n)), dim3(256), 0, s, w.w, rhs, n);
    BFX_LAUNCH_CHECK("copy_f32");
    return bfx::check_err(w, s);
}

extern "C" int bfx_ir_solve(int64_t n, const float *A, int64_t lda, const float *LU,
                            int64_t ldlu, const int32_t *ipiv, const double *b, double *x,
                            const bfx_ir_opts *opts, bfx_ir_result *res, void *ws,
                            size_t ws_bytes, void *stream) {
    bfx_ir_opts o = {1e-14, 30, 0};
    if (opts) o = *opts;
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !LU) return -4;
    if (ldlu < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !ipiv) return -6;
    if (n > 0 && !b) return -7;
    if (n > 0 && !x) return -8;
    if (!(o.tol >= 0.0) || o.max_iter < 0) return -9;
    if (!res) return -10;
    if (!ws || ws_bytes < bfx_ir_ws_size(n)) return -12;
    res->iters = 0;
    res->status = 0;
    res->eta = 0.0;
    if (n == 0) return BFX_OK;
    hipStream_t s = (hipStream_t)stream;
    bfx::IrWs w;
    bfx::ir_ws_layout(&w, ws, n);
    const unsigned g = bfx::grid_for(n);
    hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, w.err, 4);
    hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, (int32_t *)w.scal, 2 * bfx::S_NSCAL);
    hipLaunchKernelGGL(bfx::mat_norm_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, w.scal);
    hipLaunchKernelGGL(bfx::vec_absmax_kernel, dim3(g), dim3(256), 0, s, b, n, w.scal + bfx::S_NORMB);
    int rc = bfx::compose_perm(n, ipiv, w, s);
    if (rc) return rc;
    // x0 = LUsolve32(b)
    hipLaunchKernelGGL(bfx::gather_f64_to_f32, dim3(g), dim3(256), 0, s, b, w.perm, 1.0, w.w, n);
    rc = bfx::lu_solve_ws(n, LU, ldlu, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::update_x, dim3(g), dim3(256), 0, s, x, w.w, 0.0, 1, n);
    BFX_LAUNCH_CHECK("ir init");

    const int vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    unsigned long long h[bfx::S_NSCAL];
    double prev_eta = INFINITY, eta = 0.0;
    int it = 0, rises = 0, status = 1;
    for (;;) {
        hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, (int32_t *)(w.scal + bfx::S_RN), 4);
        hipLaunchKernelGGL(bfx::residual_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, b, x,
                           w.r, w.scal, vec);
        hipLaunchKernelGGL(bfx::vec_absmax_kernel, dim3(g), dim3(256), 0, s, x, n, w.scal + bfx::S_XN);
        BFX_LAUNCH_CHECK("residual");
        BFX_HIP(hipMemcpyAsync(h, w.scal, sizeof h, hipMemcpyDeviceToHost, s));
        BFX_HIP(hipStreamSynchronize(s));
        const double normA = bfx::bits_to_double(h[bfx::S_NORMA]);
        const double normb = bfx::bits_to_double(h[bfx::S_NORMB]);
        const double rn = bfx::bits_to_double(h[bfx::S_RN]);
        const double xn = bfx::bits_to_double(h[bfx::S_XN]);
        const double den = normA * xn + normb;
        eta = den > 0.0 ? rn / den : rn;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        if (!std::isfinite(eta)) { status = 3; break; }
        if (eta <= o.tol) { status = 0; break; }
        if (it >= o.max_iter) { status = 1; break; }
        if (rises >= 2) { status = 2; break; }
        hipLaunchKernelGGL(bfx::gather_f64_to_f32, dim3(g), dim3(256), 0, s, w.r, w.perm, rn,
                           w.w, n);
        rc = bfx::lu_solve_ws(n, LU, ldlu, w, s);
        if (rc) return rc;
        hipLaunchKernelGGL(bfx::update_x, dim3(g), dim3(256), 0, s, x, w.w, rn, 0, n);
        BFX_LAUNCH_CHECK("ir update");
        ++it;
    }
    res->iters = it;
    res->status = status;
    res->eta = eta;
    return bfx::check_err(w, s);
}

// ---------------------------------------------------------------------------
// GMRES-IR (Sec. III, Sec. IV-B): refinement whose correction equation is
// solved by GMRES on M^{-1} A d = M^{-1} r with M the low-precision LU,
// FP64 throughout GMRES; the preconditioner applies the FP32 factors in FP64.
// The host keeps only the O(restart) Hessenberg least-squares state (Givens
// rotations); vectors and every O(n) / O(n^2) step stay on the device.
// ---------------------------------------------------------------------------
namespace bfx {
namespace {
struct GmresWs {
    IrWs ir;
    double *V;    // (m+1) x n
    double *z;    // n
    double *h;    // 2*(m+1) + 8 scalars: hA, hB, |w|^2
    double *y;    // m
};
size_t gmres_ws_layout(GmresWs *g, void *base, int64_t n, int m) {
    size_t off = ir_ws_layout(g ? &g->ir : nullptr, base, n);
    off = (off + 255) & ~size_t(255);
    const int64_t nn = n > 0 ? n : 1;
    const size_t o_V = off; off += ((sizeof(double) * nn * (m + 1)) + 255) & ~size_t(255);
    const size_t o_z = off; off += ((sizeof(double) * nn) + 255) & ~size_t(255);
    const size_t o_h = off; off += ((sizeof(double) * (2 * (m + 1) + 8)) + 255) & ~size_t(255);
    const size_t o_y = off; off += ((sizeof(double) * (m + 1)) + 255) & ~size_t(255);
    if (g && base) {
        char *b = (char *)base;
        g->V = (double *)(b + o_V);
        g->z = (double *)(b + o_z);
        g->h = (double *)(b + o_h);
        g->y = (double *)(b + o_y);
    }
    return off;
}
}  // namespace
}  // namespace bfx

extern "C" size_t bfx_gmres_ir_ws_size(int64_t n, int restart) {
    if (restart < 1) restart = 1;
    return bfx::gmres_ws_layout(nullptr, nullptr, n < 0 ? 0 : n, restart);
}

extern "C" int bfx_gmres_ir_solve(int64_t n, const float *A, int64_t lda, const float *LU,
                                  int64_t ldlu, const int32_t *ipiv, const double *b, double *x,
                                  const bfx_gmres_opts *opts, bfx_gmres_result *res, void *ws,
                                  size_t ws_bytes, void *stream) {
    bfx_gmres_opts o = {1e-14, 30, 50, 1e-8};
    if (opts) o = *opts;
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !LU) return -4;
    if (ldlu < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !ipiv) return -6;
    if (n > 0 && !b) return -7;
    if (n > 0 && !x) return -8;
    if (!(o.tol >= 0.0) || o.max_iter < 0 || o.restart < 1 || !(o.inner_tol >= 0.0)) return -9;
    if (!res) return -10;
    const int m = o.restart;
    if (!ws || ws_bytes < bfx_gmres_ir_ws_size(n, m)) return -12;
    res->iters = 0;
    res->inner = 0;
    res->status = 0;
    res->eta = 0.0;
    if (n == 0) return BFX_OK;
    hipStream_t s = (hipStream_t)stream;
    bfx::GmresWs g;
    bfx::gmres_ws_layout(&g, ws, n, m);
    const bfx::IrWs &w = g.ir;
    const unsigned gr = bfx::grid_for(n);
    const int vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, w.err, 4);
    hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, (int32_t *)w.scal, 2 * bfx::S_NSCAL);
    hipLaunchKernelGGL(bfx::mat_norm_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, w.scal);
    hipLaunchKernelGGL(bfx::vec_absmax_kernel, dim3(gr), dim3(256), 0, s, b, n, w.scal + bfx::S_NORMB);
    int rc = bfx::compose_perm(n, ipiv, w, s);
    if (rc) return rc;
    // x0 = LUsolve32(b)
    hipLaunchKernelGGL(bfx::gather_f64_to_f32, dim3(gr), dim3(256), 0, s, b, w.perm, 1.0, w.w, n);
    rc = bfx::lu_solve_ws(n, LU, ldlu, w, s);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::update_x, dim3(gr), dim3(256), 0, s, x, w.w, 0.0, 1, n);
    BFX_LAUNCH_CHECK("gmres init");

    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), yv(m);
    std::vector<double> hh(2 * (m + 1) + 8);
    unsigned long long hs[bfx::S_NSCAL];
    double prev_eta = INFINITY, eta = 0.0;
    int it = 0, rises = 0, status = 1, inner_total = 0;
    auto precond = [&](double *v) -> int {   // v = M^{-1} v, via gather into z
        hipLaunchKernelGGL(bfx::gather_f64, dim3(gr), dim3(256), 0, s, v, w.perm, g.z, n);
        int r2 = bfx::lu_solve_vec<double>(n, LU, ldlu, g.z, w, s);
        if (r2) return r2;
        hipLaunchKernelGGL(bfx::scale_f64, dim3(gr), dim3(256), 0, s, g.z, 1.0, v, n);
        BFX_LAUNCH_CHECK("gmres precond");
        return BFX_OK;
    };
    for (;;) {
        hipLaunchKernelGGL(bfx::zero_i32, dim3(1), dim3(256), 0, s, (int32_t *)(w.scal + bfx::S_RN), 4);
        hipLaunchKernelGGL(bfx::residual_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, b, x,
                           w.r, w.scal, vec);
        hipLaunchKernelGGL(bfx::vec_absmax_kernel, dim3(gr), dim3(256), 0, s, x, n, w.scal + bfx::S_XN);
        BFX_LAUNCH_CHECK("gmres residual");
        BFX_HIP(hipMemcpyAsync(hs, w.scal, sizeof hs, hipMemcpyDeviceToHost, s));
        BFX_HIP(hipStreamSynchronize(s));
        const double normA = bfx::bits_to_double(hs[bfx::S_NORMA]);
        const double normb = bfx::bits_to_double(hs[bfx::S_NORMB]);
        const double rn = bfx::bits_to_double(hs[bfx::S_RN]);
        const double xn = bfx::bits_to_double(hs[bfx::S_XN]);
        const double den = normA * xn + normb;
        eta = den > 0.0 ? rn / den : rn;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        if (!std::isfinite(eta)) { status = 3; break; }
        if (eta <= o.tol) { status = 0; break; }
        if (it >= o.max_iter) { status = 1; break; }
        if (rises >= 2) { status = 2; break; }
        // GMRES on M^{-1} A d = M^{-1} r, d0 = 0; V_0 = M^{-1} r / beta
        rc = precond(w.r);
        if (rc) return rc;
        hipLaunchKernelGGL(bfx::dots_kernel, dim3(1), dim3(256), 0, s, w.r, n, w.r, n, g.h);
        BFX_HIP(hipMemcpyAsync(hh.data(), g.h, sizeof(double), hipMemcpyDeviceToHost, s));
        BFX_HIP(hipStreamSynchronize(s));
        const double beta = std::sqrt(hh[0]);
        int k = 0;
        if (beta > 0.0) {
            hipLaunchKernelGGL(bfx::scale_f64, dim3(gr), dim3(256), 0, s, w.r, beta, g.V, n);
            std::fill(gv.begin(), gv.end(), 0.0);
            gv[0] = beta;
            for (k = 0; k < m; ++k) {
                double *vk = g.V + (int64_t)k * n;
                double *wv = w.r;   // the residual is recomputed next step: reuse as w
                hipLaunchKernelGGL(bfx::matvec_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n,
                                   vk, wv, vec);
                rc = precond(wv);
                if (rc) return rc;
                double *hA = g.h, *hB = g.h + (m + 1), *nw = g.h + 2 * (m + 1);
                hipLaunchKernelGGL(bfx::dots_kernel, dim3(k + 1), dim3(256), 0, s, g.V, n, wv, n, hA);
                hipLaunchKernelGGL(bfx::combine_kernel, dim3(gr), dim3(256), 0, s, g.V, n, hA, k + 1,
                                   wv, n, -1.0);
                hipLaunchKernelGGL(bfx::dots_kernel, dim3(k + 1), dim3(256), 0, s, g.V, n, wv, n, hB);
                hipLaunchKernelGGL(bfx::combine_kernel, dim3(gr), dim3(256), 0, s, g.V, n, hB, k + 1,
                                   wv, n, -1.0);
                hipLaunchKernelGGL(bfx::dots_kernel, dim3(1), dim3(256), 0, s, wv, n, wv, n, nw);
                BFX_LAUNCH_CHECK("gmres arnoldi");
                BFX_HIP(hipMemcpyAsync(hh.data(), g.h, sizeof(double) * (2 * (m + 1) + 1),
                                       hipMemcpyDeviceToHost, s));
                BFX_HIP(hipStreamSynchronize(s));
                const double hn = std::sqrt(hh[2 * (m + 1)]);
                for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = hh[j] + hh[(m + 1) + j];
                H[(size_t)(k + 1) * m + k] = hn;
                for (int j = 0; j < k; ++j) {
                    const double a = H[(size_t)j * m + k], c2 = H[(size_t)(j + 1) * m + k];
                    H[(size_t)j * m + k] = cs[j] * a + sn[j] * c2;
                    H[(size_t)(j + 1) * m + k] = -sn[j] * a + cs[j] * c2;
                }
                const double a = H[(size_t)k * m + k], c2 = H[(size_t)(k + 1) * m + k];
                const double rho = std::hypot(a, c2);
                cs[k] = rho > 0.0 ? a / rho : 1.0;
                sn[k] = rho > 0.0 ? c2 / rho : 0.0;
                H[(size_t)k * m + k] = rho;
                H[(size_t)(k + 1) * m + k] = 0.0;
                gv[k + 1] = -sn[k] * gv[k];
                gv[k] = cs[k] * gv[k];
                ++inner_total;
                if (hn > 0.0)
                    hipLaunchKernelGGL(bfx::scale_f64, dim3(gr), dim3(256), 0, s, wv, hn,
                                       g.V + (int64_t)(k + 1) * n, n);
                if (std::fabs(gv[k + 1]) <= o.inner_tol * beta || hn == 0.0) { ++k; break; }
            }
            for (int j = k - 1; j >= 0; --j) {
                double acc = gv[j];
                for (int q = j + 1; q < k; ++q) acc -= H[(size_t)j * m + q] * yv[q];
                yv[j] = acc / H[(size_t)j * m + j];
            }
            BFX_HIP(hipMemcpyAsync(g.y, yv.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(bfx::combine_kernel, dim3(gr), dim3(256), 0, s, g.V, n, g.y, k, x, n, 1.0);
            BFX_LAUNCH_CHECK("gmres update");
            BFX_HIP(hipStreamSynchronize(s));
        }
        ++it;
    }
    res->iters = it;
    res->inner = inner_total;
    res->status = status;
    res->eta = eta;
    return bfx::check_err(w, s);
}
