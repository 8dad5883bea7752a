// Iterative refinement in residual form (Sec. III), GMRES-IR (Sec. III,
// Sec. IV-B) and the FP32 LU solve.
//
//   x0 = LUsolve32(b);  repeat: r = b - A x (FP64, A promoted exactly),
//   eta = |r|_inf / (|A|_inf |x|_inf + |b|_inf), stop when eta <= tol;
//   LU-IR:    s = |r|_inf, d = s * LUsolve32(r / s), x += d (FP64);
//   GMRES-IR: d from GMRES on M^-1 A d = M^-1 r (FP64, M = the FP32 factors
//             applied in FP64 arithmetic), x += d.
//
// Only the cubic LU is low precision; every quadratic step is FP64 except the
// FP32 triangular solves of LU-IR.
//
// Device residency.  A solve is one stream of kernels that the host queues
// without waiting: the convergence test runs on the device (ir_check_kernel)
// and writes the caller's bfx_ir_result / bfx_gmres_result in device memory;
// once it decides to stop, it sets a flag that every later kernel of the
// solve reads first and returns on.  The host therefore queues the largest
// possible number of steps (max_iter corrections, and `restart` GMRES steps
// per correction); the steps after convergence cost one empty launch each.
// GMRES keeps its Hessenberg least-squares problem on the device as well
// (givens_kernel applies the rotations, backsolve_kernel solves R y = g).
//
// Kernels:
//   residual_kernel  one workgroup per row, FP64 FMA, |r|_inf by atomicMax on
//                    the bit pattern of a non-negative double (order-free);
//   trsv_kernel      blocked triangular solve without a global barrier: each
//                    workgroup takes the next block row from a ticket counter,
//                    adds the contributions of the blocks it depends on as
//                    their solution values arrive, solves its 128 x 128
//                    diagonal block in one wave and publishes the values as
//                    64-bit words tagged with the number of the launch, so
//                    that a reader needs neither a flag nor a fence and no
//                    launch has to clear the words for the next;
//   perm_kernel      the row permutation of ipiv, composed once per solve
//                    (every position evaluated in parallel);
//   GMRES            matvec_perm_kernel (P A v, materialising the basis
//                    vector), dots_kernel / combine_kernel (classical
//                    Gram-Schmidt applied twice), givens_kernel,
//                    backsolve_kernel, update with the basis.
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
constexpr int CROWS = 64;                  // rows per workgroup of the basis kernels

enum { S_NORMA = 0, S_NORMB = 1, S_RN = 2, S_XN = 3, S_NSCAL = 8 };

// Refinement state in device memory.
struct IrCtrl {
    int32_t done;      // refinement finished: every later kernel returns at once
    int32_t iters;     // corrections applied (or about to be)
    int32_t status;
    int32_t rises;     // consecutive checks whose eta did not decrease
    int32_t inner;     // GMRES steps in total
    int32_t k;         // basis vectors of the current GMRES cycle
    int32_t gdone;     // the current GMRES cycle has finished
    int32_t err;       // a bounded wait expired
    double eta, prev_eta;
    double rn;         // |r|_inf of the current residual
    double beta;       // GMRES: |M^-1 r|_2 at the start of the cycle
    double rinv;       // GMRES: 1 / norm of the next basis vector
    double pad;
};

struct IrWs {
    int32_t *perm;
    float *w;
    double *r;
    uint64_t *xch;    // [2n] tagged solution words exchanged between workgroups
    uint32_t *ticket; // [4]
    unsigned long long *scal;  // [S_NSCAL]
    IrCtrl *ctrl;
    double *part;     // [ceil(n / CROWS)]
};

size_t ir_ws_layout(IrWs *w, void *base, int64_t n) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const int64_t nn = n > 0 ? n : 1;
    const size_t o_perm = take(sizeof(int32_t) * nn);
    const size_t o_w = take(sizeof(float) * nn);
    const size_t o_r = take(sizeof(double) * nn);
    const size_t o_f = take(sizeof(uint64_t) * 2 * nn);
    const size_t o_t = take(sizeof(uint32_t) * 4);
    const size_t o_s = take(sizeof(unsigned long long) * S_NSCAL);
    const size_t o_c = take(sizeof(IrCtrl));
    const size_t o_p = take(sizeof(double) * ceil_div(nn, CROWS));
    if (w && base) {
        char *b = (char *)base;
        w->perm = (int32_t *)(b + o_perm);
        w->w = (float *)(b + o_w);
        w->r = (double *)(b + o_r);
        w->xch = (uint64_t *)(b + o_f);
        w->ticket = (uint32_t *)(b + o_t);
        w->scal = (unsigned long long *)(b + o_s);
        w->ctrl = (IrCtrl *)(b + o_c);
        w->part = (double *)(b + o_p);
    }
    return off;
}

// A kernel of the solve returns at once when the refinement has stopped, and
// a kernel of a GMRES step (inner = 1) also when the current cycle has.
__device__ __forceinline__ bool stopped(const IrCtrl *c, int inner) {
    return c && (c->done || (inner && c->gdone));
}
}  // namespace

__device__ __forceinline__ void atomic_max_abs(unsigned long long *dst, double v) {
    // |v| as a non-negative double orders like its bit pattern (NaN above Inf)
    atomicMax(dst, (unsigned long long)__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ double bits_double(unsigned long long u) { return __longlong_as_double((long long)u); }

// Start of a solve: clear the exchange words, tickets, reduction scalars and
// the control block; the caller's result says "not converged" until a check
// runs.
__global__ void __launch_bounds__(256)
ir_begin_kernel(IrCtrl *c, unsigned long long *scal, uint32_t *ticket, uint64_t *xch, int64_t nx) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nx; i += (int64_t)gridDim.x * 256) xch[i] = 0ull;
    if (blockIdx.x != 0) return;
    if (threadIdx.x < 4) ticket[threadIdx.x] = 0u;
    if (threadIdx.x < S_NSCAL) scal[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        IrCtrl z;
        z.done = 0; z.iters = 0; z.status = 1; z.rises = 0;
        z.inner = 0; z.k = 0; z.gdone = 1; z.err = 0;
        z.eta = 0.0; z.prev_eta = INFINITY; z.rn = 1.0; z.beta = 0.0; z.rinv = 0.0; z.pad = 0.0;
        *c = z;
    }
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
    extern __shared__ __align__(16) int32_t sp[];
    const int32_t *iv = ipiv;
    if (use_lds) {
        for (int64_t i = threadIdx.x; i < n; i += 256) sp[i] = ipiv[i];
        __syncthreads();
        iv = sp;
    }
    const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pos >= n) return;
    int32_t p = (int32_t)pos;
    int32_t i = (int32_t)n - 1;
    if (use_lds) {
        // 16-byte LDS reads of four interchanges at a time, several in
        // flight (every lane reads the same address: a broadcast)
        for (; i >= 0 && (i & 3) != 3; --i) {
            const int32_t q = iv[i];
            p = (p == i) ? q : ((p == q) ? i : p);
        }
        const int4 *iv4 = reinterpret_cast<const int4 *>(sp);
#pragma unroll 8
        for (int32_t ch = (i + 1) / 4 - 1; ch >= 0; --ch) {
            const int4 q = iv4[ch];
            const int32_t b = 4 * ch;
            p = (p == b + 3) ? q.w : ((p == q.w) ? b + 3 : p);
            p = (p == b + 2) ? q.z : ((p == q.z) ? b + 2 : p);
            p = (p == b + 1) ? q.y : ((p == q.y) ? b + 1 : p);
            p = (p == b) ? q.x : ((p == q.x) ? b : p);
        }
    } else {
        for (; i >= 0; --i) {
            const int32_t q = iv[i];
            p = (p == i) ? q : ((p == q) ? i : p);
        }
    }
    perm[pos] = p;
}

// w[i] = (float)(src[perm[i]] / div), div = 1 or the current |r|_inf.
__global__ void __launch_bounds__(256)
gather_f64_to_f32(const double *src, const int32_t *perm, const IrCtrl *c, int use_rn, float *w, int64_t n) {
    if (stopped(c, 0)) return;
    const double div = use_rn ? c->rn : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = (float)(src[perm[i]] / div);
}

__global__ void __launch_bounds__(256)
gather_f32(const float *src, const int32_t *perm, float *w, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = src[perm[i]];
}

__global__ void __launch_bounds__(256)
gather_f64(const double *src, const int32_t *perm, double *out, int64_t n, const IrCtrl *c) {
    if (stopped(c, 0)) return;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = src[perm[i]];
}

__global__ void __launch_bounds__(256) copy_f32(const float *src, float *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

// x = (double) w   (init)   or   x += |r|_inf * (double) w   (update)
__global__ void __launch_bounds__(256)
update_x(double *x, const float *w, const IrCtrl *c, int init, int64_t n) {
    if (stopped(c, 0)) return;
    const double s = c->rn;
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

// Sum_j A[row, j] * (v[j] * scale), A promoted exactly, fixed-order reduction
// over the workgroup (every thread gets the sum).
__device__ __forceinline__ double row_dot(const float *a, int64_t n, const double *v, double scale, int vec,
                                          double *red) {
    double s = 0.0;
    if (vec) {
        for (int64_t j = 4 * threadIdx.x; j + 3 < n; j += 1024) {
            const float4 q = *reinterpret_cast<const float4 *>(a + j);
            s = fma((double)q.x, v[j] * scale, s);
            s = fma((double)q.y, v[j + 1] * scale, s);
            s = fma((double)q.z, v[j + 2] * scale, s);
            s = fma((double)q.w, v[j + 3] * scale, s);
        }
        for (int64_t j = (n & ~int64_t(3)) + threadIdx.x; j < n; j += 256) s = fma((double)a[j], v[j] * scale, s);
    } else {
        for (int64_t j = threadIdx.x; j < n; j += 256) s = fma((double)a[j], v[j] * scale, s);
    }
    return block_sum_256(s, red);
}

// r_i = b_i - sum_j A_ij x_j in FP64; |r|_inf into scal[S_RN].
__global__ void __launch_bounds__(256)
residual_kernel(const float *A, int64_t lda, int64_t n, const double *b, const double *x,
                double *r, unsigned long long *scal, int vec, const IrCtrl *c) {
    __shared__ double red[4];
    if (stopped(c, 0)) return;
    const int64_t row = blockIdx.x;
    const double s = row_dot(A + row * lda, n, x, 1.0, vec, red);
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
vec_absmax_kernel(const double *v, int64_t n, unsigned long long *dst, const IrCtrl *c) {
    if (stopped(c, 0)) return;
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

// The convergence test of check number `check` (0-based, = corrections
// applied so far), one thread: eta from the reduced norms, then the stopping
// rule; writes the caller's result, and either stops the solve or clears the
// reductions for the next residual.  Status: 0 converged, 1 max_iter
// reached, 2 stagnated (eta did not decrease twice in a row), 3 non-finite,
// 4 a bounded wait expired.
__global__ void __launch_bounds__(64)
ir_check_kernel(IrCtrl *c, unsigned long long *scal, bfx_ir_result *res, bfx_gmres_result *gres,
                double tol, int max_iter) {
    if (threadIdx.x != 0 || c->done) return;
    const double normA = bits_double(scal[S_NORMA]);
    const double normb = bits_double(scal[S_NORMB]);
    const double rn = bits_double(scal[S_RN]);
    const double xn = bits_double(scal[S_XN]);
    const double den = normA * xn + normb;
    const double eta = den > 0.0 ? rn / den : rn;
    const int rises = (eta >= c->prev_eta) ? c->rises + 1 : 0;
    c->rises = rises;
    c->prev_eta = eta;
    c->eta = eta;
    c->rn = rn;
    int st = -1;
    if (c->err) st = 4;
    else if (!(eta <= INFINITY) || eta == INFINITY) st = 3;
    else if (eta <= tol) st = 0;
    else if (c->iters >= max_iter) st = 1;
    else if (rises >= 2) st = 2;
    if (res) {
        res->iters = c->iters;
        res->status = st >= 0 ? st : 1;
        res->eta = eta;
    }
    if (gres) {
        gres->iters = c->iters;
        gres->inner = c->inner;
        gres->status = st >= 0 ? st : 1;
        gres->reserved = 0;
        gres->eta = eta;
    }
    if (st >= 0) {
        c->status = st;
        c->done = 1;
        return;
    }
    c->iters += 1;     // the correction queued next is applied
    c->k = 0;
    c->gdone = 0;
    scal[S_RN] = 0ull;
    scal[S_XN] = 0ull;
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

// Solution values travel between workgroups as 64-bit words that carry the
// number of the launch that wrote them (the epoch) in their upper half: one
// word per FP32 value, two (high and low half) per FP64 value.  A word is
// written and read whole, so a reader that sees its launch's epoch in every
// word of a value has the value, without a flag, a fence or a second read.
template <typename T> struct Xch;
template <> struct Xch<float> {
    static constexpr int W = 1;
    __device__ static void put(uint64_t *x, int64_t i, float v, uint32_t tag) {
        __hip_atomic_store(x + i, ((uint64_t)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static float value(const uint64_t *w) { return __uint_as_float((uint32_t)w[0]); }
};
template <> struct Xch<double> {
    static constexpr int W = 2;
    __device__ static void put(uint64_t *x, int64_t i, double v, uint32_t tag) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        __hip_atomic_store(x + 2 * i, ((uint64_t)tag << 32) | (u >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(x + 2 * i + 1, ((uint64_t)tag << 32) | (u & 0xffffffffull), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static double value(const uint64_t *w) {
        return __longlong_as_double((long long)(((w[0] & 0xffffffffull) << 32) | (w[1] & 0xffffffffull)));
    }
};

// Blocked triangular solve with the FP32 LU factors, in place on y; T is the
// arithmetic and vector type (float for LU-IR, double for the GMRES
// preconditioner).  lower = 1: unit lower L (forward); lower = 0: upper U
// (backward, divides).  One workgroup per block row of TB = 128 rows, taken in
// dependency order from a ticket counter.  Off-diagonal part: wave w owns rows
// 16w .. 16w+15 of the block row as 8 row pairs; for every dependency block
// each half-wave reads one row of a pair with 16-byte loads (4 consecutive
// columns per lane, 512 bytes per half-wave) and accumulates per row in
// column order, the row sums being reduced across the half-wave at the end.
// The factor values and exchange words of the next two dependencies are in
// flight while the current one is used, which keeps enough bytes in flight
// per workgroup for the dependency sweep to run ahead of the chain of block
// solves.  A wave whose words of a block do not carry this launch's epoch
// yet polls them again (bounded).  Diagonal block: one wave, lane l holding
// rows l and l + 64, substitution in column order with the diagonal block in
// LDS; the results go to y and, tagged, to the exchange words.
//
// `epoch` numbers the launches of one solve (1, 2, ...); launch e takes its
// tickets from ticket[e % 3] and clears ticket[(e + 1) % 3] for the launch
// after it (the launch before it, which used that counter, has completed in
// stream order).  vec = 1: LU and ld allow 16-byte loads.
template <typename T>
__global__ void __launch_bounds__(512)
trsv_kernel(const float *LU, int64_t ld, int64_t n, T *y, uint64_t *xch, uint32_t *ticket,
            int32_t epoch, int32_t *err, const IrCtrl *c, int inner, int lower, int vec) {
    extern __shared__ float Ld[];   // [TB][TB + 1] diagonal block
    __shared__ int s_blk;
    __shared__ T rhs[TB];
    constexpr int LDD = TB + 1;
    constexpr int W = Xch<T>::W;
    constexpr int NX = 4 * W;       // exchange words of a lane's 4 columns
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int half = lane >> 5, hl = lane & 31;
    if (blockIdx.x == 0 && t == 0) ticket[(epoch + 1) % 3] = 0u;
    if (stopped(c, inner)) return;
    const uint32_t tag = (uint32_t)epoch;
    const int64_t nblk = ceil_div(n, TB);
    if (t == 0) s_blk = (int)atomicAdd(ticket + epoch % 3, 1u);
    __syncthreads();
    const int64_t blk = lower ? s_blk : nblk - 1 - s_blk;
    const int64_t r0 = blk * TB;
    const int rows = (int)((n - r0 < TB) ? n - r0 : TB);
    // diagonal block to LDS (independent of other blocks)
    for (int e = t; e < TB * TB; e += 512) {
        const int i = e / TB, cc = e % TB;
        Ld[i * LDD + cc] = (i < rows && cc < rows) ? LU[(r0 + i) * ld + r0 + cc] : 0.0f;
    }
    const int64_t nb_dep = lower ? blk : nblk - 1 - blk;
    // row 16 wave + 2 p + half of this block row (clamped: rows past the end
    // of the matrix re-read the last row and are never stored)
    const float *lrow[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int rr = 16 * wave + 2 * p + half;
        lrow[p] = LU + (r0 + (rr < rows ? rr : rows - 1)) * ld;
    }
    auto col0 = [&](int64_t d) { return (lower ? d : nblk - 1 - d) * TB + 4 * hl; };
    struct Stage {
        float4 l[8];
        uint64_t x[NX];
    };
    auto load = [&](Stage &st, int64_t col) {
        if (vec && col + 3 < n) {
#pragma unroll
            for (int p = 0; p < 8; ++p) st.l[p] = *reinterpret_cast<const float4 *>(lrow[p] + col);
        } else {
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                st.l[p].x = (col < n) ? lrow[p][col] : 0.0f;
                st.l[p].y = (col + 1 < n) ? lrow[p][col + 1] : 0.0f;
                st.l[p].z = (col + 2 < n) ? lrow[p][col + 2] : 0.0f;
                st.l[p].w = (col + 3 < n) ? lrow[p][col + 3] : 0.0f;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < W; ++h)
                st.x[q * W + h] = (col + q < n)
                                      ? __hip_atomic_load(xch + (col + q) * W + h, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : ((uint64_t)tag << 32);
    };
    auto reload_x = [&](Stage &st, int64_t col) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int h = 0; h < W; ++h)
                st.x[q * W + h] = (col + q < n)
                                      ? __hip_atomic_load(xch + (col + q) * W + h, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : ((uint64_t)tag << 32);
    };
    auto present = [&](const Stage &st) {
        bool ok = true;
#pragma unroll
        for (int i = 0; i < NX; ++i) ok = ok && (uint32_t)(st.x[i] >> 32) == tag;
        return ok;
    };
    // this block's right-hand side, read before the sweep (it is not on the
    // chain of block solves)
    T yown = 0;
    if (hl < 8) {
        const int rr = 16 * wave + 2 * hl + half;
        if (rr < rows) yown = y[r0 + rr];
    }
    T acc[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) acc[p] = 0;
    Stage s0, s1, s2;
    if (nb_dep > 0) load(s0, col0(0));
    if (nb_dep > 1) load(s1, col0(1));
    for (int64_t d = 0; d < nb_dep; ++d) {
        if (d + 2 < nb_dep) load(s2, col0(d + 2));
        unsigned spins = 0;
        while (!__all(present(s0))) {
            // another workgroup's expired wait is checked every 256 polls
            if ((++spins & 255u) == 0 &&
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                break;
            if (spins > SPIN_LIMIT) { atomicExch(err, 1); break; }
            __builtin_amdgcn_s_sleep(1);
            reload_x(s0, col0(d));
        }
        const T y0 = Xch<T>::value(s0.x), y1 = Xch<T>::value(s0.x + W);
        const T y2 = Xch<T>::value(s0.x + 2 * W), y3 = Xch<T>::value(s0.x + 3 * W);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            acc[p] = fma((T)s0.l[p].x, y0, acc[p]);
            acc[p] = fma((T)s0.l[p].y, y1, acc[p]);
            acc[p] = fma((T)s0.l[p].z, y2, acc[p]);
            acc[p] = fma((T)s0.l[p].w, y3, acc[p]);
        }
        s0 = s1;
        s1 = s2;
    }
#pragma unroll
    for (int p = 0; p < 8; ++p)
        for (int off = 16; off > 0; off >>= 1) acc[p] += __shfl_xor(acc[p], off);
    if (hl < 8) {
        // lane hl of each half publishes row 16 wave + 2 hl + half (static
        // register index via a select chain)
        T v = acc[0];
#pragma unroll
        for (int p = 1; p < 8; ++p) if (hl == p) v = acc[p];
        const int rr = 16 * wave + 2 * hl + half;
        if (rr < rows) rhs[rr] = yown - v;
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
                    const int cc = 8 * ch + k;
                    const T yc = bcast_lane(cc < 64 ? v0 : v1, cc & 63);
                    const T u0 = fma(-(T)a0[k], yc, v0), u1 = fma(-(T)a1[k], yc, v1);
                    v0 = (lane > cc) ? u0 : v0;
                    v1 = (lane + 64 > cc) ? u1 : v1;
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
                    const int cc = 8 * ch + k;
                    if (cc < rows) {
                        const T yc = bcast_lane(cc < 64 ? v0 : v1, cc & 63);
                        const T u0 = fma(-((T)a0[k] * rd0), yc, v0), u1 = fma(-((T)a1[k] * rd1), yc, v1);
                        v0 = (lane < cc) ? u0 : v0;
                        v1 = (lane + 64 < cc) ? u1 : v1;
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) { a0[k] = b0[k]; a1[k] = b1[k]; }
            }
        }
        if (lane < rows) {
            Xch<T>::put(xch, r0 + lane, v0, tag);
            y[r0 + lane] = v0;
        }
        if (lane + 64 < rows) {
            Xch<T>::put(xch, r0 + 64 + lane, v1, tag);
            y[r0 + 64 + lane] = v1;
        }
    }
}


// ---------------------------------------------------------------------------
// GMRES pieces (all FP64 vectors).
// ---------------------------------------------------------------------------
// z[i] = (P A v)[i] = sum_j A[perm[i], j] v[j] with v = w * rinv, the next
// basis vector, which workgroup i also stores: V_k[i] = w[i] * rinv (the
// product the dot product uses, so the stored vector is the one multiplied).
__global__ void __launch_bounds__(256)
matvec_perm_kernel(const float *A, int64_t lda, int64_t n, const int32_t *perm, const double *w,
                   double *Vk, double *z, int vec, const IrCtrl *c) {
    __shared__ double red[4];
    if (stopped(c, 1)) return;
    const int64_t i = blockIdx.x;
    const double rinv = c->rinv;
    const double s = row_dot(A + (int64_t)perm[i] * lda, n, w, rinv, vec, red);
    if (threadIdx.x == 0) {
        z[i] = s;
        Vk[i] = w[i] * rinv;
    }
}

// h[j] = <V_j, z>, j < gridDim.x: one workgroup per j, fixed-order tree.
__global__ void __launch_bounds__(256)
dots_kernel(const double *V, int64_t ldv, const double *z, int64_t n, double *h, const IrCtrl *c) {
    __shared__ double red[4];
    if (stopped(c, 1)) return;
    const double *v = V + (int64_t)blockIdx.x * ldv;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s = fma(v[i], z[i], s);
    s = block_sum_256(s, red);
    if (threadIdx.x == 0) h[blockIdx.x] = s;
}

// out[i] = z[i] + sign * sum_{j < cnt} h[j] V_j[i] over CROWS = 64 rows per
// workgroup: lane = row, wave q sums j = q, q + 4, ... in increasing j, the
// four wave sums are added in a fixed order (deterministic).  cnt < 0 takes
// the count from the control block (the basis size of the finished cycle);
// part != NULL also stores the workgroup's sum of out^2.  inner selects the
// gate (a Gram-Schmidt pass of a GMRES step, or the update of x).
__global__ void __launch_bounds__(256)
combine_kernel(const double *V, int64_t ldv, const double *h, int cnt, const double *z, double *out,
               int64_t n, double sign, double *part, const IrCtrl *c, int inner) {
    __shared__ double red[4][CROWS];
    if (stopped(c, inner)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * CROWS + lane;
    const int k = cnt >= 0 ? cnt : c->k;
    double s = 0.0;
    if (i < n) {
        int j = wave;
        for (; j + 12 < k; j += 16) {
            const double v0 = V[(int64_t)j * ldv + i], v1 = V[(int64_t)(j + 4) * ldv + i];
            const double v2 = V[(int64_t)(j + 8) * ldv + i], v3 = V[(int64_t)(j + 12) * ldv + i];
            s = fma(h[j], v0, s);
            s = fma(h[j + 4], v1, s);
            s = fma(h[j + 8], v2, s);
            s = fma(h[j + 12], v3, s);
        }
        for (; j < k; j += 4) s = fma(h[j], V[(int64_t)j * ldv + i], s);
    }
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0) {
        double o = 0.0;
        if (i < n) {
            const double tot = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
            o = fma(sign, tot, z[i]);
            out[i] = o;
        }
        if (part) {
            double q = o * o;
            for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
            if (lane == 0) part[blockIdx.x] = q;
        }
    }
}

// part[blockIdx] = sum of v[i]^2 over the workgroup's CROWS rows.
__global__ void __launch_bounds__(64)
nrm_part_kernel(const double *v, int64_t n, double *part, const IrCtrl *c) {
    if (stopped(c, 0)) return;
    const int64_t i = (int64_t)blockIdx.x * CROWS + threadIdx.x;
    double q = (i < n) ? v[i] * v[i] : 0.0;
    for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off);
    if (threadIdx.x == 0) part[blockIdx.x] = q;
}

// Sum of the partials in a fixed order (one wave; every lane gets it).
__device__ __forceinline__ double sum_parts(const double *part, int64_t np) {
    double s = 0.0;
    for (int64_t p = threadIdx.x; p < np; p += 64) s += part[p];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

// Start of a GMRES cycle on w = M^-1 r: beta = |w|_2, g = beta e_1.
__global__ void __launch_bounds__(64)
gmres_begin_kernel(IrCtrl *c, const double *part, int64_t np, double *g) {
    if (stopped(c, 0)) return;
    const double beta = sqrt(sum_parts(part, np));
    if (threadIdx.x == 0) {
        c->beta = beta;
        c->k = 0;
        c->gdone = (beta > 0.0 && beta < INFINITY) ? 0 : 1;
        c->rinv = 1.0 / beta;
        g[0] = beta;
    }
}

// Step k of the cycle after Gram-Schmidt: column k of the Hessenberg matrix
// is h_j = hA_j + hB_j (j <= k), h_{k+1} = |w|_2; the k earlier rotations are
// applied to it in order, a new rotation zeroes h_{k+1}, and the rotated
// column is stored as column k of R (column-major, leading dimension m).
// One wave: the rotations form a chain, walked 64 at a time with the
// rotation and column values of a chunk loaded in parallel, one per lane,
// and broadcast with v_readlane.  The cycle ends when |g_{k+1}| <= inner_tol
// * beta, when the new vector is zero or when the basis is full.
__global__ void __launch_bounds__(64)
givens_kernel(IrCtrl *c, const double *hA, const double *hB, const double *part, int64_t np, double *R,
              int m, double *cs, double *sn, double *g, double inner_tol) {
    if (stopped(c, 1)) return;
    const int lane = threadIdx.x;
    const int k = c->k;
    const double hn = sqrt(sum_parts(part, np));
    double *col = R + (int64_t)k * m;
    // carry: the column entry j after rotations 0 .. j-1
    double carry = hA[0] + hB[0];
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + lane;
        const double cj = (j < k) ? cs[j] : 1.0, sj = (j < k) ? sn[j] : 0.0;
        const double hnext = (j < k) ? hA[j + 1] + hB[j + 1] : 0.0;
        double outv = 0.0;
        const int cnt = (k - j0 < 64) ? k - j0 : 64;
        for (int l = 0; l < cnt; ++l) {
            const double cl = bcast_lane(cj, l), sl = bcast_lane(sj, l), hl = bcast_lane(hnext, l);
            const double top = cl * carry + sl * hl;
            carry = -sl * carry + cl * hl;
            outv = (lane == l) ? top : outv;
        }
        if (j < k) col[j] = outv;
    }
    if (lane == 0) {
        const double a = carry, b2 = hn;
        const double rho = hypot(a, b2);
        const double ck = rho > 0.0 ? a / rho : 1.0, sk = rho > 0.0 ? b2 / rho : 0.0;
        cs[k] = ck;
        sn[k] = sk;
        col[k] = rho;
        const double gk = g[k];
        g[k + 1] = -sk * gk;
        g[k] = ck * gk;
        const int kk = k + 1;
        c->k = kk;
        c->inner += 1;
        c->rinv = 1.0 / hn;
        const bool conv = fabs(g[kk]) <= inner_tol * c->beta || hn == 0.0;
        c->gdone = (conv || kk >= m) ? 1 : 0;
    }
}

// y = R^-1 g for the k x k upper triangle of the finished cycle, column by
// column from the last (g is overwritten).
__global__ void __launch_bounds__(256)
backsolve_kernel(const IrCtrl *c, const double *R, int m, double *g, double *y) {
    __shared__ double s_y;
    if (stopped(c, 0)) return;
    const int k = c->k;
    for (int j = k - 1; j >= 0; --j) {
        if (threadIdx.x == 0) {
            const double v = g[j] / R[(int64_t)j * m + j];
            y[j] = v;
            s_y = v;
        }
        __syncthreads();
        const double yj = s_y;
        const double *colj = R + (int64_t)j * m;
        for (int i = threadIdx.x; i < j; i += 256) g[i] = fma(-colj[i], yj, g[i]);
        __syncthreads();
    }
}

static unsigned grid_for(int64_t n) {
    int64_t b = ceil_div(n, 256);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// One solve's launches: the trsv epoch counter and the shared arguments.
struct Solver {
    int64_t n;
    const float *LU;
    int64_t ldlu;
    IrWs w;
    hipStream_t s;
    int32_t epoch = 0;

    template <typename T>
    int trsv_pair(T *y, const IrCtrl *c, int inner) {
        const int vec = ((uintptr_t)LU % 16 == 0) && (ldlu % 4 == 0);
        static bool attr = false;
        if (!attr) {
            BFX_HIP(hipFuncSetAttribute((const void *)trsv_kernel<T>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)TRSV_LDS));
            attr = true;
        }
        const int64_t nb = ceil_div(n, TB);
        for (int lower = 1; lower >= 0; --lower) {
            ++epoch;
            hipLaunchKernelGGL(trsv_kernel<T>, dim3((unsigned)nb), dim3(512), TRSV_LDS, s, LU, ldlu, n, y,
                               w.xch, w.ticket, epoch, &w.ctrl->err, c, inner, lower, vec);
            BFX_LAUNCH_CHECK("trsv_kernel");
        }
        return BFX_OK;
    }

    int compose_perm(const int32_t *ipiv) {
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
        hipLaunchKernelGGL(perm_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), use_lds ? lds : 0, s, ipiv,
                           n, w.perm, use_lds);
        BFX_LAUNCH_CHECK("perm_kernel");
        return BFX_OK;
    }

    // Clear the state, norms of A and b, the permutation and
    // x0 = (double) LUsolve32((float) b).
    int begin(const float *A, int64_t lda, const int32_t *ipiv, const double *b, double *x) {
        const unsigned g = grid_for(n);
        hipLaunchKernelGGL(ir_begin_kernel, dim3(grid_for(2 * n)), dim3(256), 0, s, w.ctrl, w.scal, w.ticket,
                           w.xch, 2 * n);
        hipLaunchKernelGGL(mat_norm_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, w.scal);
        hipLaunchKernelGGL(vec_absmax_kernel, dim3(g), dim3(256), 0, s, b, n, w.scal + S_NORMB,
                           (const IrCtrl *)nullptr);
        int rc = compose_perm(ipiv);
        if (rc) return rc;
        hipLaunchKernelGGL(gather_f64_to_f32, dim3(g), dim3(256), 0, s, b, w.perm, w.ctrl, 0, w.w, n);
        rc = trsv_pair<float>(w.w, w.ctrl, 0);
        if (rc) return rc;
        hipLaunchKernelGGL(update_x, dim3(g), dim3(256), 0, s, x, w.w, w.ctrl, 1, n);
        BFX_LAUNCH_CHECK("refinement start");
        return BFX_OK;
    }

    // r = b - A x, |x|_inf and the convergence test.
    int check(const float *A, int64_t lda, int vec, const double *b, const double *x, bfx_ir_result *res,
              bfx_gmres_result *gres, double tol, int max_iter) {
        hipLaunchKernelGGL(residual_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, b, x, w.r, w.scal, vec,
                           w.ctrl);
        hipLaunchKernelGGL(vec_absmax_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, w.scal + S_XN, w.ctrl);
        hipLaunchKernelGGL(ir_check_kernel, dim3(1), dim3(64), 0, s, w.ctrl, w.scal, res, gres, tol, max_iter);
        BFX_LAUNCH_CHECK("refinement check");
        return BFX_OK;
    }
};

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
    bfx::Solver sv{n, LU, ldlu, {}, s};
    bfx::ir_ws_layout(&sv.w, ws, n);
    hipLaunchKernelGGL(bfx::ir_begin_kernel, dim3(bfx::grid_for(2 * n)), dim3(256), 0, s, sv.w.ctrl, sv.w.scal,
                       sv.w.ticket, sv.w.xch, 2 * n);
    int rc = sv.compose_perm(ipiv);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::gather_f32, dim3(bfx::grid_for(n)), dim3(256), 0, s, rhs, sv.w.perm, sv.w.w, n);
    rc = sv.trsv_pair<float>(sv.w.w, sv.w.ctrl, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(bfx::copy_f32, dim3(bfx::grid_for(n)), dim3(256), 0, s, sv.w.w, rhs, n);
    BFX_LAUNCH_CHECK("copy_f32");
    // The only synchronisation of this utility: report an expired bounded wait.
    int32_t e = 0;
    BFX_HIP(hipMemcpyAsync(&e, &sv.w.ctrl->err, sizeof e, hipMemcpyDeviceToHost, s));
    BFX_HIP(hipStreamSynchronize(s));
    if (e) {
        bfx::set_error("triangular solve: a bounded wait on a block flag expired");
        return BFX_E_INTERNAL;
    }
    return BFX_OK;
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
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        const bfx_ir_result z = {0, 0, 0.0};
        BFX_HIP(hipMemcpyAsync(res, &z, sizeof z, hipMemcpyHostToDevice, s));
        return BFX_OK;
    }
    bfx::Solver sv{n, LU, ldlu, {}, s};
    bfx::ir_ws_layout(&sv.w, ws, n);
    const bfx::IrWs &w = sv.w;
    const unsigned g = bfx::grid_for(n);
    const int vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    int rc = sv.begin(A, lda, ipiv, b, x);
    if (rc) return rc;
    for (int it = 0;; ++it) {
        rc = sv.check(A, lda, vec, b, x, res, nullptr, o.tol, o.max_iter);
        if (rc) return rc;
        if (it >= o.max_iter) break;
        // d = |r|_inf LUsolve32(r / |r|_inf), x += d
        hipLaunchKernelGGL(bfx::gather_f64_to_f32, dim3(g), dim3(256), 0, s, w.r, w.perm, w.ctrl, 1, w.w, n);
        rc = sv.trsv_pair<float>(w.w, w.ctrl, 0);
        if (rc) return rc;
        hipLaunchKernelGGL(bfx::update_x, dim3(g), dim3(256), 0, s, x, w.w, w.ctrl, 0, n);
        BFX_LAUNCH_CHECK("ir update");
    }
    return BFX_OK;
}

// ---------------------------------------------------------------------------
// GMRES-IR (Sec. III, Sec. IV-B): refinement whose correction equation is
// solved by GMRES on M^{-1} A d = M^{-1} r with M the low-precision LU,
// FP64 throughout GMRES; the preconditioner applies the FP32 factors in FP64.
// ---------------------------------------------------------------------------
namespace bfx {
namespace {
struct GmresWs {
    IrWs ir;
    double *V;    // (m+1) x n basis
    double *z;    // n
    double *wv;   // n: the vector the next basis vector is made from
    double *hA, *hB;   // m+1 each: the two Gram-Schmidt passes
    double *R;    // m x m, column-major: rotated Hessenberg columns
    double *cs, *sn;   // m each
    double *g;    // m+1
    double *y;    // m
};
size_t gmres_ws_layout(GmresWs *g, void *base, int64_t n, int m) {
    size_t off = ir_ws_layout(g ? &g->ir : nullptr, base, n);
    const int64_t nn = n > 0 ? n : 1;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_V = take(sizeof(double) * nn * (size_t)(m + 1));
    const size_t o_z = take(sizeof(double) * nn);
    const size_t o_w = take(sizeof(double) * nn);
    const size_t o_hA = take(sizeof(double) * (m + 1));
    const size_t o_hB = take(sizeof(double) * (m + 1));
    const size_t o_R = take(sizeof(double) * (size_t)m * (size_t)m);
    const size_t o_cs = take(sizeof(double) * m);
    const size_t o_sn = take(sizeof(double) * m);
    const size_t o_g = take(sizeof(double) * (m + 1));
    const size_t o_y = take(sizeof(double) * m);
    if (g && base) {
        char *b = (char *)base;
        g->V = (double *)(b + o_V);
        g->z = (double *)(b + o_z);
        g->wv = (double *)(b + o_w);
        g->hA = (double *)(b + o_hA);
        g->hB = (double *)(b + o_hB);
        g->R = (double *)(b + o_R);
        g->cs = (double *)(b + o_cs);
        g->sn = (double *)(b + o_sn);
        g->g = (double *)(b + o_g);
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
    bfx_gmres_opts o = {1e-14, 10, 50, 1e-8};
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
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        const bfx_gmres_result z = {0, 0, 0, 0, 0.0};
        BFX_HIP(hipMemcpyAsync(res, &z, sizeof z, hipMemcpyHostToDevice, s));
        return BFX_OK;
    }
    bfx::GmresWs gw;
    bfx::gmres_ws_layout(&gw, ws, n, m);
    bfx::Solver sv{n, LU, ldlu, gw.ir, s};
    const bfx::IrWs &w = sv.w;
    bfx::IrCtrl *c = w.ctrl;
    const unsigned gr = bfx::grid_for(n);
    const unsigned gc = (unsigned)bfx::ceil_div(n, bfx::CROWS);
    const int vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
    int rc = sv.begin(A, lda, ipiv, b, x);
    if (rc) return rc;
    for (int it = 0;; ++it) {
        rc = sv.check(A, lda, vec, b, x, nullptr, res, o.tol, o.max_iter);
        if (rc) return rc;
        if (it >= o.max_iter) break;
        // wv = M^-1 r = U^-1 L^-1 P r, beta = |wv|_2
        hipLaunchKernelGGL(bfx::gather_f64, dim3(gr), dim3(256), 0, s, w.r, w.perm, gw.wv, n, c);
        rc = sv.trsv_pair<double>(gw.wv, c, 0);
        if (rc) return rc;
        hipLaunchKernelGGL(bfx::nrm_part_kernel, dim3(gc), dim3(64), 0, s, gw.wv, n, w.part, c);
        hipLaunchKernelGGL(bfx::gmres_begin_kernel, dim3(1), dim3(64), 0, s, c, w.part, (int64_t)gc, gw.g);
        BFX_LAUNCH_CHECK("gmres begin");
        for (int k = 0; k < m; ++k) {
            double *Vk = gw.V + (int64_t)k * n;
            // z = M^-1 A v_k with v_k = wv / |wv|_2 stored as V_k
            hipLaunchKernelGGL(bfx::matvec_perm_kernel, dim3((unsigned)n), dim3(256), 0, s, A, lda, n, w.perm,
                               gw.wv, Vk, gw.z, vec, c);
            rc = sv.trsv_pair<double>(gw.z, c, 1);
            if (rc) return rc;
            // classical Gram-Schmidt, twice; the second pass writes wv and |wv|^2
            hipLaunchKernelGGL(bfx::dots_kernel, dim3(k + 1), dim3(256), 0, s, gw.V, n, gw.z, n, gw.hA, c);
            hipLaunchKernelGGL(bfx::combine_kernel, dim3(gc), dim3(256), 0, s, gw.V, n, gw.hA, k + 1, gw.z, gw.z,
                               n, -1.0, (double *)nullptr, c, 1);
            hipLaunchKernelGGL(bfx::dots_kernel, dim3(k + 1), dim3(256), 0, s, gw.V, n, gw.z, n, gw.hB, c);
            hipLaunchKernelGGL(bfx::combine_kernel, dim3(gc), dim3(256), 0, s, gw.V, n, gw.hB, k + 1, gw.z, gw.wv,
                               n, -1.0, w.part, c, 1);
            hipLaunchKernelGGL(bfx::givens_kernel, dim3(1), dim3(64), 0, s, c, gw.hA, gw.hB, w.part, (int64_t)gc,
                               gw.R, m, gw.cs, gw.sn, gw.g, o.inner_tol);
            BFX_LAUNCH_CHECK("gmres step");
        }
        // d = V y with R y = g; x += d
        hipLaunchKernelGGL(bfx::backsolve_kernel, dim3(1), dim3(256), 0, s, c, gw.R, m, gw.g, gw.y);
        hipLaunchKernelGGL(bfx::combine_kernel, dim3(gc), dim3(256), 0, s, gw.V, n, gw.y, -1, x, x, n, 1.0,
                           (double *)nullptr, c, 0);
        BFX_LAUNCH_CHECK("gmres update");
    }
    return BFX_OK;
}
