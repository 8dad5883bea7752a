// Many independent dense solves A x = b (n <= 1024) in one persistent,
// graph-captured launch: split-BF16 blocked LU (Sec. I, IV-A) followed by
// FP64-residual iterative refinement (Sec. III), and GMRES-IR (Sec. III,
// Sec. IV-B) for the systems that LU-IR leaves unconverged, one workgroup per
// problem.
//
// Per problem, inside one 256-thread workgroup:
//   LU     panels of 32 columns held in LDS (pivot search by wave shuffles and
//          LDS, swap, divide, rank-1 update), the panel's interchanges on
//          the other columns (composed once, applied column by column through
//          LDS), TRSM with L11 in LDS, and the trailing update
//          A22 -= L21 U12 as a rank-32 split-BF16 update on the four waves
//          (alpha = -1, beta = 1; rank32_update);
//   IR     |A|_inf and |b|_inf, the permutation from ipiv, then
//          x0 = LUsolve32(b) and refinement steps with an FP64 residual (one
//          wave per row) and FP32 triangular solves in 64-row blocks (the
//          diagonal block in LDS, solved by one wave);
//   GMRES  when LU-IR stops without converging (max_iter reached or
//          stagnation) and GMRES is enabled: refinement from x0 again (a
//          stalled or diverging LU-IR can leave x where GMRES-IR stalls too)
//          with FP64 GMRES on M^-1 A d = M^-1 r, M the FP32 factors applied
//          in FP64 arithmetic, classical Gram-Schmidt twice, Givens
//          rotations; the basis and the rotated Hessenberg matrix live in the
//          workgroup's slice of the plan's scratch, the vectors in LDS.
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
constexpr int SWP_OFF = 0;       // int offset of the interchange lists (after the panel's write-back)

struct SolveItem {
    int64_t n;
    const float *A;
    int64_t lda;
    const double *b;
    double *x;
    float *LU;        // n x n, leading dimension n
    int32_t *ipiv;
    bfx_gmres_result *res;
    int32_t *info;
};

// GMRES fallback settings shared by the launch.
struct GmresCfg {
    int lu_format;     // 0: split-BF16 blocked LU; 1, 2: single-format BF16, FP16 LU
    int mode;          // 0: LU-IR (GMRES-IR if it fails); 1: GMRES-IR from the start
    int max_iter;      // refinement steps with GMRES (0: no fallback)
    int restart;       // basis size per cycle (0: n, a full Krylov space)
    double inner_tol;  // relative GMRES tolerance
    int64_t m_cap;     // basis capacity of a workgroup's scratch slice
    double *scratch;   // gridDim.x slices of per_wg doubles
    int64_t per_wg;
};

// LDS byte offsets of the refinement phases (inside the LU panel's space).
constexpr int L_Y = 0;          // n floats (LU-IR solve vector)
constexpr int L_R = 4096;       // n doubles: residual
constexpr int L_PERM = 12288;   // n ints: row permutation
constexpr int L_D = 16384;      // 64 x 65 floats: diagonal block of a solve
constexpr int L_V = 33024;      // n doubles: current basis vector
constexpr int L_W = 41216;      // n doubles: GMRES work vector
constexpr int L_HA = 49408;     // m + 1 doubles: first Gram-Schmidt pass
constexpr int L_HB = 57608;     // m + 1 doubles: second pass
constexpr int L_CS = 65808;     // m doubles: rotation cosines
constexpr int L_SN = 74000;     // m doubles: rotation sines
constexpr int L_G = 82192;      // m + 1 doubles: rotated right-hand side
constexpr int L_END = 90392;
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

// a pointer the whole wave holds, made explicitly uniform (so that buffer
// resources built from it live in scalar registers)
__device__ __forceinline__ float *uniform_ptr(float *p) {
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (float *)(((uint64_t)hi << 32) | lo);
}

// Buffer resource over len floats from p (p uniform over the wave).  Loads
// at a byte offset of len*4 or more return 0 and stores there are dropped, so
// a loop can issue all its loads before the first use without a branch per
// element: an element past the end takes an out-of-range offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const float *p, int len) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(const_cast<float *>(p)), (short)0, len * 4,
                                             0x00020000);
}
constexpr int OOB = 0x40000000;   // a byte offset past every span here

// In-place solve of (L or U) y = y with y in LDS (T = float for LU-IR, double
// for the GMRES preconditioner), FP32 factors in global LU.
template <typename T, bool LOWER>
__device__ void block_trsv(const float *LU, int n, T *y, float *D) {
    const int t = threadIdx.x, lane = t & 63;
    const int nblk = (n + STB - 1) / STB;
    for (int bb = 0; bb < nblk; ++bb) {
        const int blk = LOWER ? bb : nblk - 1 - bb;
        const int k0 = blk * STB;
        const int rows = (n - k0 < STB) ? n - k0 : STB;
        {
            // the diagonal block: a thread's 16 loads in flight before their
            // LDS stores (entries outside it load as 0)
            const __amdgpu_buffer_rsrc_t rd = span_rsrc(LU + (int64_t)k0 * n + k0, (rows - 1) * n + rows);
            float v[STB * STB / 256];
#pragma unroll
            for (int k = 0; k < STB * STB / 256; ++k) {
                const int e = t + 256 * k, i = e / STB, c = e % STB;
                v[k] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(rd, (i < rows && c < rows) ? (i * n + c) * 4 : OOB, 0, 0));
            }
#pragma unroll
            for (int k = 0; k < STB * STB / 256; ++k) {
                const int e = t + 256 * k, i = e / STB, c = e % STB;
                D[i * (STB + 1) + c] = v[k];
            }
        }
        __syncthreads();
        if (t < 64) {
            T v = (lane < rows) ? y[k0 + lane] : (T)0;
            if (LOWER) {
                for (int c = 0; c < rows; ++c) {
                    const T yc = __shfl(v, c);
                    if (lane > c) v = fma(-(T)D[lane * (STB + 1) + c], yc, v);
                }
            } else {
                for (int c = rows - 1; c >= 0; --c) {
                    if (lane == c) v = v / (T)D[c * (STB + 1) + c];
                    const T yc = __shfl(v, c);
                    if (lane < c) v = fma(-(T)D[lane * (STB + 1) + c], yc, v);
                }
            }
            if (lane < rows) y[k0 + lane] = v;
        }
        __syncthreads();
        // update the rows not yet solved with this block's solution
        const int lo = LOWER ? k0 + rows : 0, hi = LOWER ? n : k0;
        if (rows == STB) {
            // whole 64-column block: sixteen 16-byte loads per row, all in
            // flight (buffer loads: rows need only 4-byte alignment)
            const __amdgpu_buffer_rsrc_t rl = span_rsrc(LU, n * n);
            for (int i = lo + t; i < hi; i += 256) {
                const int ro = (i * n + k0) * 4;
                float4 a[16];
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    a[q] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rl, ro + 16 * q, 0, 0));
                T acc = (T)0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    acc = fma((T)a[q].x, y[k0 + 4 * q], acc);
                    acc = fma((T)a[q].y, y[k0 + 4 * q + 1], acc);
                    acc = fma((T)a[q].z, y[k0 + 4 * q + 2], acc);
                    acc = fma((T)a[q].w, y[k0 + 4 * q + 3], acc);
                }
                y[i] -= acc;
            }
        } else {
            for (int i = lo + t; i < hi; i += 256) {
                const float *row = LU + (int64_t)i * n + k0;
                T acc = (T)0;
                for (int c = 0; c < rows; ++c) acc = fma((T)row[c], y[k0 + c], acc);
                y[i] -= acc;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double block_sum_d(double v, double *sd) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sd[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = (sd[0] + sd[1]) + (sd[2] + sd[3]);
    __syncthreads();
    return s;
}

// Row dot products of one workgroup, out[row] = sum_c A[src(row)][c] u[c]
// (u in LDS, n <= 1024): each wave takes two rows at a time, each lane
// four columns per 256-column chunk, so that every lane has eight 16-byte
// loads in flight before the first FMA (rows one at a time with one load
// per FMA wait for memory at every step).  src(row) = perm[row] when perm
// is given.  Accumulation per lane in column order, then a wave reduction.
__device__ void rowdots_wg(const float *A, int64_t lda, int n, const int32_t *perm, const double *u,
                           double *out, int vec) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int row0 = 2 * wave; row0 < n; row0 += 8) {
        float4 a[2][4];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int row = row0 + rr < n ? row0 + rr : n - 1;
            const float *ar = A + (int64_t)(perm ? perm[row] : row) * lda;
            if (vec) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 4 * lane + 256 * q;
                    if (c + 3 < n) {
                        a[rr][q] = *reinterpret_cast<const float4 *>(ar + c);
                    } else {
                        a[rr][q].x = (c < n) ? ar[c] : 0.0f;
                        a[rr][q].y = (c + 1 < n) ? ar[c + 1] : 0.0f;
                        a[rr][q].z = (c + 2 < n) ? ar[c + 2] : 0.0f;
                        a[rr][q].w = (c + 3 < n) ? ar[c + 3] : 0.0f;
                    }
                }
            } else {
                // rows without 16-byte alignment: 4-byte buffer loads, all in
                // flight, entries past n by an out-of-range offset (load 0)
                const __amdgpu_buffer_rsrc_t ra = span_rsrc(ar, n);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 4 * lane + 256 * q;
                    float v[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        v[e] = __uint_as_float(
                            __builtin_amdgcn_raw_buffer_load_b32(ra, c + e < n ? (c + e) * 4 : OOB, 0, 0));
                    a[rr][q] = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
        }
        double sacc[2] = {0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * lane + 256 * q;
            const double u0 = (c < n) ? u[c] : 0.0, u1 = (c + 1 < n) ? u[c + 1] : 0.0;
            const double u2 = (c + 2 < n) ? u[c + 2] : 0.0, u3 = (c + 3 < n) ? u[c + 3] : 0.0;
#pragma unroll
            for (int rr = 0; rr < 2; ++rr) {
                sacc[rr] = fma((double)a[rr][q].x, u0, sacc[rr]);
                sacc[rr] = fma((double)a[rr][q].y, u1, sacc[rr]);
                sacc[rr] = fma((double)a[rr][q].z, u2, sacc[rr]);
                sacc[rr] = fma((double)a[rr][q].w, u3, sacc[rr]);
            }
        }
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            double v = sacc[rr];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0 && row0 + rr < n) out[row0 + rr] = v;
        }
    }
}

// h[j] = <V_j, w> for j = 0 .. k (V_j: n doubles in global memory, w in
// LDS): each wave takes two basis vectors at a time with all of a lane's
// loads (16 per vector for n = 1024) issued before its FMAs.
__device__ void basis_dots_wg(const double *V, int n, int k, const double *w, double *h) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j0 = 2 * wave; j0 <= k; j0 += 8) {
        double x[2][16];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const double *vj = V + (int64_t)(j0 + jj <= k ? j0 + jj : k) * n;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = lane + 64 * q;
                x[jj][q] = (i < n) ? vj[i] : 0.0;
            }
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            double sacc = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = lane + 64 * q;
                if (i < n) sacc = fma(x[jj][q], w[i], sacc);
            }
            for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
            if (lane == 0 && j0 + jj <= k) h[j0 + jj] = sacc;
        }
    }
}

// out[i] = base[i] + sign * sum_{j < cnt} h[j] V_j[i] for i < n: each thread
// takes its (up to four) rows together and four basis vectors per step, so
// that sixteen loads are in flight.
__device__ void basis_combine_wg(const double *V, int n, int cnt, const double *h, const double *base,
                                 double *out, double sign) {
    const int t = threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 3 < cnt; j += 4) {
        double x[4][4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = t + 256 * q;
                x[jj][q] = (i < n) ? V[(int64_t)(j + jj) * n + i] : 0.0;
            }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(h[j + jj], x[jj][q], acc[q]);
    }
    for (; j < cnt; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = t + 256 * q;
            if (i < n) acc[q] = fma(h[j], V[(int64_t)j * n + i], acc[q]);
        }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = t + 256 * q;
        if (i < n) out[i] = fma(sign, acc[q], base[i]);
    }
}

// r = b - A x (FP64) into LDS, x staged in LDS at xs; returns |r|_inf.
__device__ double residual_wg(const SolveItem &it, int n, double *r, double *xs, double *sd) {
    const int t = threadIdx.x;
    for (int i = t; i < n; i += 256) xs[i] = it.x[i];
    __syncthreads();
    const int vec = ((uintptr_t)it.A % 16 == 0) && (it.lda % 4 == 0);
    rowdots_wg(it.A, it.lda, n, nullptr, xs, r, vec);
    __syncthreads();
    double rl = 0.0;
    for (int i = t; i < n; i += 256) {
        const double ri = it.b[i] - r[i];
        r[i] = ri;
        const double a = fabs(ri);
        if (a > rl || a != a) rl = a;
    }
    return block_max_d(rl, sd);
}

__device__ double absmax_x_wg(const SolveItem &it, int n, double *sd) {
    double xl = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double a = fabs(it.x[i]);
        if (a > xl || a != a) xl = a;
    }
    return block_max_d(xl, sd);
}

// The stopping rule of the refinement (status as bfx_ir_result; -1: go on).
__device__ __forceinline__ int ir_decide(double eta, double tol, int iters, int max_iter, int rises) {
    if (!(eta <= INFINITY) || eta == INFINITY) return 3;
    if (eta <= tol) return 0;
    if (iters >= max_iter) return 1;
    if (rises >= 2) return 2;
    return -1;
}

// GMRES-IR from the current x (Sec. III, Sec. IV-B): each refinement step
// solves A d = r by one GMRES cycle on M^-1 A d = M^-1 r (d0 = 0), M = the
// FP32 factors applied in FP64; x += d.  Returns the status; adds the
// refinement and GMRES steps taken to iters and inner; eta is the last one.
__device__ int gmres_phase(const SolveItem &it, const GmresCfg &cfg, double normA, double normb, double tol,
                           uint16_t *smem, int &iters, int &inner, double &eta) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n = (int)it.n;
    const float *LU = it.LU;
    char *sb = reinterpret_cast<char *>(smem);
    double *r = reinterpret_cast<double *>(sb + L_R);
    const int32_t *perm = reinterpret_cast<const int32_t *>(sb + L_PERM);
    float *D = reinterpret_cast<float *>(sb + L_D);
    double *v = reinterpret_cast<double *>(sb + L_V);
    double *w = reinterpret_cast<double *>(sb + L_W);
    double *hA = reinterpret_cast<double *>(sb + L_HA);
    double *hB = reinterpret_cast<double *>(sb + L_HB);
    double *cs = reinterpret_cast<double *>(sb + L_CS);
    double *sn = reinterpret_cast<double *>(sb + L_SN);
    double *g = reinterpret_cast<double *>(sb + L_G);
    __shared__ double s_d[4];
    __shared__ double s_hn;
    __shared__ int s_conv;
    const int m = (int)((cfg.restart > 0 && cfg.restart < n) ? cfg.restart : n);
    double *V = cfg.scratch + (int64_t)blockIdx.x * cfg.per_wg;          // (m_cap + 1) x n
    double *R = V + (cfg.m_cap + 1) * (int64_t)n;                         // m_cap x m_cap, column-major
    const int64_t ldr = cfg.m_cap;
    const int avec = ((uintptr_t)it.A % 16 == 0) && (it.lda % 4 == 0);
    int steps = 0, rises = 0, status = 1;
    double prev_eta = INFINITY;
    for (;;) {
        const double rn = residual_wg(it, n, r, v, s_d);
        const double xn = absmax_x_wg(it, n, s_d);
        const double den = normA * xn + normb;
        eta = den > 0.0 ? rn / den : rn;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        status = ir_decide(eta, tol, steps, cfg.max_iter, rises);
        if (status >= 0) break;
        // w = M^-1 r = U^-1 L^-1 P r
        for (int i = t; i < n; i += 256) w[i] = r[perm[i]];
        __syncthreads();
        block_trsv<double, true>(LU, n, w, D);
        block_trsv<double, false>(LU, n, w, D);
        double q = 0.0;
        for (int i = t; i < n; i += 256) q = fma(w[i], w[i], q);
        const double beta = sqrt(block_sum_d(q, s_d));
        int k = 0;
        if (beta > 0.0 && beta < INFINITY) {
            const double rb = 1.0 / beta;
            for (int i = t; i < n; i += 256) {
                const double vi = w[i] * rb;
                v[i] = vi;
                V[i] = vi;
            }
            if (t == 0) g[0] = beta;
            __syncthreads();
            for (k = 0; k < m;) {
                // w = P A v
                rowdots_wg(it.A, it.lda, n, perm, v, w, avec);
                __syncthreads();
                block_trsv<double, true>(LU, n, w, D);
                block_trsv<double, false>(LU, n, w, D);
                // classical Gram-Schmidt, twice
                for (int pass = 0; pass < 2; ++pass) {
                    double *h = pass ? hB : hA;
                    basis_dots_wg(V, n, k, w, h);
                    __syncthreads();
                    basis_combine_wg(V, n, k + 1, h, w, w, -1.0);
                    __syncthreads();
                }
                double qq = 0.0;
                for (int i = t; i < n; i += 256) qq = fma(w[i], w[i], qq);
                const double hn = sqrt(block_sum_d(qq, s_d));
                if (t == 0) {
                    // earlier rotations on column k, then a new one
                    double *col = R + (int64_t)k * ldr;
                    double carry = hA[0] + hB[0];
                    for (int j = 0; j < k; ++j) {
                        const double hj1 = hA[j + 1] + hB[j + 1];
                        col[j] = cs[j] * carry + sn[j] * hj1;
                        carry = -sn[j] * carry + cs[j] * hj1;
                    }
                    const double rho = hypot(carry, hn);
                    const double ck = rho > 0.0 ? carry / rho : 1.0, sk = rho > 0.0 ? hn / rho : 0.0;
                    cs[k] = ck;
                    sn[k] = sk;
                    col[k] = rho;
                    const double gk = g[k];
                    g[k + 1] = -sk * gk;
                    g[k] = ck * gk;
                    s_conv = (fabs(g[k + 1]) <= cfg.inner_tol * beta || hn == 0.0) ? 1 : 0;
                    s_hn = hn;
                }
                __syncthreads();
                ++k;
                ++inner;
                if (s_conv || k >= m) break;
                const double rh = 1.0 / s_hn;
                double *Vk = V + (int64_t)k * n;
                for (int i = t; i < n; i += 256) {
                    const double vi = w[i] * rh;
                    v[i] = vi;
                    Vk[i] = vi;
                }
                __syncthreads();
            }
            // y = R^-1 g (column by column from the last; y in hA), x += V y
            double *y = hA;
            for (int j = k - 1; j >= 0; --j) {
                if (t == 0) y[j] = g[j] / R[(int64_t)j * ldr + j];
                __syncthreads();
                const double yj = y[j];
                const double *colj = R + (int64_t)j * ldr;
                for (int i = t; i < j; i += 256) g[i] = fma(-colj[i], yj, g[i]);
                __syncthreads();
            }
            basis_combine_wg(V, n, k, y, it.x, it.x, 1.0);
            __syncthreads();
        }
        ++steps;
    }
    iters += steps;
    return status;
}

// Round an exact FP64 value once to the single format of the LU (1: BF16,
// 2: FP16): nearest even, gradual underflow, overflow to Inf.
__device__ __forceinline__ double round_fmt(double x, int fmt) {
    const int p = fmt == 1 ? 8 : 11;
    const int emin = fmt == 1 ? -126 : -14, emax = fmt == 1 ? 127 : 15;
    if (x == 0.0 || !(fabs(x) < INFINITY)) return x;
    int e;
    (void)frexp(x, &e);   // |x| in [2^(e-1), 2^e)
    e -= 1;
    if (e < emin) e = emin;
    const double q = ldexp(1.0, e - p + 1);
    const double r = rint(x / q) * q;
    if (fabs(r) >= ldexp(1.0, emax + 1)) return copysign((double)INFINITY, x);
    return r;
}

// Single-format LU (the BF16 and FP16 rows of the Sec. IV-B tables), in
// place on the factor storage that holds a copy of A: every entry rounded to
// the format, then elimination with partial pivoting in which every
// multiplier and every update is rounded to the format once (the update as a
// fused multiply-add: l u + a is exact in FP64 for these formats).
__device__ void lu_fmt_wg(const SolveItem &it, int fmt, float *s_v, int *s_i) {
    const int t = threadIdx.x;
    const int n = (int)it.n;
    float *LU = it.LU;
    for (int64_t e = t; e < (int64_t)n * n; e += 256) LU[e] = (float)round_fmt((double)LU[e], fmt);
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        float bv = -1.0f;
        int bi = INT_MAX;
        for (int r = c + t; r < n; r += 256) {
            float v = fabsf(LU[(int64_t)r * n + c]);
            if (!(v == v)) v = INFINITY;
            argmax_better(bv, bi, v, r);
        }
        block_argmax(bv, bi, s_v, s_i);
        const int p = bi;
        if (t == 0) {
            it.ipiv[c] = p;
            if (LU[(int64_t)p * n + c] == 0.0f && *it.info == 0) *it.info = c + 1;
        }
        if (p != c)
            for (int q = t; q < n; q += 256) {
                const float x = LU[(int64_t)c * n + q];
                LU[(int64_t)c * n + q] = LU[(int64_t)p * n + q];
                LU[(int64_t)p * n + q] = x;
            }
        __syncthreads();
        const double piv = LU[(int64_t)c * n + c];
        if (piv == 0.0) continue;   // uniform: the column below is zero
        for (int r = c + 1 + t; r < n; r += 256)
            LU[(int64_t)r * n + c] = (float)round_fmt((double)LU[(int64_t)r * n + c] / piv, fmt);
        __syncthreads();
        const int m = n - c - 1;
        for (int e = t; e < m * m; e += 256) {
            const int r = c + 1 + e / m, q = c + 1 + e % m;
            const double l = LU[(int64_t)r * n + c];
            LU[(int64_t)r * n + q] =
                (float)round_fmt(fma(-l, (double)LU[(int64_t)c * n + q], (double)LU[(int64_t)r * n + q]), fmt);
        }
        __syncthreads();
    }
}

// A22 -= L21 U12 for one problem's trailing matrix when the panel is a full
// 32 columns (K = 32, rest x rest), on the workgroup's four waves without
// barriers: wave w takes the 32 x 32 output blocks w, w + 4, ... in
// row-major order.  Each lane loads its MFMA fragments' FP32 values (A row
// lane % 16 and B column lane % 16, k = 8 (lane / 16) .. + 7) and its C values
// straight into registers through buffer loads, splits them there and runs
// the products; the next block's values are loaded while the current block
// computes.  Elements outside the trailing matrix get an offset beyond the
// buffer, so they load as zero and their stores are dropped, without
// branches.  Zero padding, split, product order (lo products in the listed
// order, then hi) and epilogue are the general tile engine's, so the result
// is the same bits.
struct Rank32Frag {
    float a[2][8], b[2][8], c[2][2][4];
};
constexpr uint32_t R32_OOR = 0x80000000u;   // beyond every buffer's range

// VEC: the A fragment's 8 values by two 16-byte loads instead of eight
// 4-byte loads (buffer loads need only 4-byte alignment here: measured the
// same bits for odd n), which keeps a block's loads and stores within what
// the wave's memory counter tells apart.
template <bool VEC>
__device__ __forceinline__ void rank32_load(__amdgpu_buffer_rsrc_t rL, __amdgpu_buffer_rsrc_t rU,
                                            __amdgpu_buffer_rsrc_t rC, int n, int rest, int nb, int blk,
                                            int r16, int kg, Rank32Frag &f) {
    const int m0 = (blk / nb) * 32, n0 = (blk % nb) * 32;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int row = m0 + i * 16 + r16, col = n0 + i * 16 + r16;
        const uint32_t oa = row < rest ? (uint32_t)(row * n + kg * 8) * 4u : R32_OOR;
        const uint32_t ob = col < rest ? (uint32_t)(kg * 8 * n + col) * 4u : R32_OOR;
        if constexpr (VEC) {
            const bfx_f32x4 v0 = __builtin_bit_cast(bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rL, oa, 0, 0));
            const bfx_f32x4 v1 =
                __builtin_bit_cast(bfx_f32x4, __builtin_amdgcn_raw_buffer_load_b128(rL, oa + 16u, 0, 0));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                f.a[i][e] = v0[e];
                f.a[i][4 + e] = v1[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                f.a[i][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rL, oa + 4u * e, 0, 0));
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
            f.b[i][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rU, ob + 4u * n * e, 0, 0));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + i * 16 + kg * 4 + e, col = n0 + jj * 16 + r16;
                const uint32_t oc = (row < rest && col < rest) ? (uint32_t)(row * n + col) * 4u : R32_OOR;
                f.c[i][jj][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rC, oc, 0, 0));
            }
}

template <int V>
__device__ __forceinline__ void rank32_compute(__amdgpu_buffer_rsrc_t rC, int n, int rest, int nb, int blk,
                                               int r16, int kg, const Rank32Frag &f) {
    using PR = Prods<V>;
    constexpr int P = PR::P;
    const int m0 = (blk / nb) * 32, n0 = (blk % nb) * 32;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    bfx_bf16x8 af[P][2], bf[P][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        uint32_t h0[3][2], h1[3][2], g0[3][2], g1[3][2];
        split4<P>(&f.a[i][0], h0);
        split4<P>(&f.a[i][4], h1);
        split4<P>(&f.b[i][0], g0);
        split4<P>(&f.b[i][4], g1);
#pragma unroll
        for (int pl = 0; pl < P; ++pl) {
            af[pl][i] = __builtin_bit_cast(bfx_bf16x8, u32x4{h0[pl][0], h0[pl][1], h1[pl][0], h1[pl][1]});
            bf[pl][i] = __builtin_bit_cast(bfx_bf16x8, u32x4{g0[pl][0], g0[pl][1], g1[pl][0], g1[pl][1]});
        }
    }
    bfx_f32x4 hi[2][2], lo[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            hi[i][jj] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
            lo[i][jj] = bfx_f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
    for (int q = 0; q < PR::n; ++q)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
                lo[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[PR::ai[q]][i], bf[PR::bj[q]][jj], lo[i][jj],
                                                                    0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
            hi[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[0][jj], hi[i][jj], 0, 0, 0);
    // the epilogue of the general engine with alpha = -1, beta = 1
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + i * 16 + kg * 4 + e, col = n0 + jj * 16 + r16;
                const uint32_t oc = (row < rest && col < rest) ? (uint32_t)(row * n + col) * 4u : R32_OOR;
                const float x = fmaf(-1.0f, hi[i][jj][e] + lo[i][jj][e], 1.0f * f.c[i][jj][e]);
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), rC, oc, 0, 0);
            }
}



template <int V, bool VEC>
__device__ __forceinline__ void rank32_update(float *LU_, int n_, int j_, int rest_) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    float *LU = uniform_ptr(LU_);
    const int n = __builtin_amdgcn_readfirstlane(n_), j = __builtin_amdgcn_readfirstlane(j_);
    const int rest = __builtin_amdgcn_readfirstlane(rest_);
    float *L21 = LU + (int64_t)(j + 32) * n + j;
    float *U12 = LU + (int64_t)j * n + j + 32;
    float *C = LU + (int64_t)(j + 32) * n + j + 32;
    const __amdgpu_buffer_rsrc_t rL =
        __builtin_amdgcn_make_buffer_rsrc((void *)L21, (short)0, ((rest - 1) * n + 32) * 4, 0x00020000);
    const __amdgpu_buffer_rsrc_t rU =
        __builtin_amdgcn_make_buffer_rsrc((void *)U12, (short)0, (31 * n + rest) * 4, 0x00020000);
    const __amdgpu_buffer_rsrc_t rC =
        __builtin_amdgcn_make_buffer_rsrc((void *)C, (short)0, ((rest - 1) * n + rest) * 4, 0x00020000);
    const int nb = (rest + 31) / 32, total = nb * nb;
    // two blocks in flight ahead of the one being computed
    Rank32Frag f0, f1, f2;
    int b = wave;
    if (b < total) rank32_load<VEC>(rL, rU, rC, n, rest, nb, b, r16, kg, f0);
    if (b + 4 < total) rank32_load<VEC>(rL, rU, rC, n, rest, nb, b + 4, r16, kg, f1);
    while (b < total) {
        if (b + 8 < total) rank32_load<VEC>(rL, rU, rC, n, rest, nb, b + 8, r16, kg, f2);
        rank32_compute<V>(rC, n, rest, nb, b, r16, kg, f0);
        b += 4;
        if (b >= total) break;
        if (b + 8 < total) rank32_load<VEC>(rL, rU, rC, n, rest, nb, b + 8, r16, kg, f0);
        rank32_compute<V>(rC, n, rest, nb, b, r16, kg, f1);
        b += 4;
        if (b >= total) break;
        if (b + 8 < total) rank32_load<VEC>(rL, rU, rC, n, rest, nb, b + 8, r16, kg, f1);
        rank32_compute<V>(rC, n, rest, nb, b, r16, kg, f2);
        b += 4;
    }
}

template <int V>
__device__ __forceinline__ void solve_one(const SolveItem &it, double tol, int max_iter, const GmresCfg &cfg,
                                          uint16_t *smem) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n = (int)it.n;
    float *LU = it.LU;
    __shared__ float s_v[4];
    __shared__ int s_i[4];
    __shared__ double s_d[4];

    // ---- copy A into the factor storage: a wave per row, lanes along it,
    // 8 loads in flight before their stores
    for (int r = wave; r < n; r += 4) {
        const __amdgpu_buffer_rsrc_t rs = span_rsrc(it.A + (int64_t)r * it.lda, n);
        const __amdgpu_buffer_rsrc_t rd = span_rsrc(LU + (int64_t)r * n, n);
        for (int c0 = 0; c0 < n; c0 += 512) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = c0 + lane + 64 * k;
                v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, c < n ? c * 4 : OOB, 0, 0));
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = c0 + lane + 64 * k;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[k]), rd, c < n ? c * 4 : OOB, 0, 0);
            }
        }
    }
    if (t == 0) *it.info = 0;
    __syncthreads();

    // ---- LU: single-format, or blocked with split-GEMM trailing updates
    if (cfg.lu_format) lu_fmt_wg(it, cfg.lu_format, s_v, s_i);
    for (int j = 0; j < (cfg.lu_format ? 0 : n); j += SNB) {
        const int jb = (n - j < SNB) ? n - j : SNB;
        const int m = n - j;
        float *P = reinterpret_cast<float *>(smem);
        {
            // 8 loads in flight per thread before their LDS stores
            const __amdgpu_buffer_rsrc_t rp = span_rsrc(LU + (int64_t)j * n + j, (m - 1) * n + jb);
            for (int e0 = 0; e0 < m * SNB; e0 += 8 * 256) {
                float v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + 256 * k + t, r = e >> 5, q = e & (SNB - 1);
                    v[k] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(rp, (r < m && q < jb) ? (r * n + q) * 4 : OOB, 0, 0));
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + 256 * k + t, r = e >> 5, q = e & (SNB - 1);
                    if (r < m && q < jb) P[r * SLD + q] = v[k];
                }
            }
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
            if (jb == SNB) {
                // whole rows through registers: all of a row's LDS reads issue
                // before its FMAs (columns q <= c are written back unchanged,
                // then column c receives the multiplier)
                float u[SNB];
#pragma unroll
                for (int q = 0; q < SNB; ++q) u[q] = P[c * SLD + q];
                for (int r = c + 1 + t; r < m; r += 256) {
                    float x[SNB];
#pragma unroll
                    for (int q = 0; q < SNB; ++q) x[q] = P[r * SLD + q];
                    float l = P[r * SLD + c];
                    if (piv != 0.0f) l = l / piv;
#pragma unroll
                    for (int q = 0; q < SNB; ++q) {
                        const float y = fmaf(-l, u[q], x[q]);
                        x[q] = q > c ? y : x[q];
                    }
#pragma unroll
                    for (int q = 0; q < SNB; ++q) P[r * SLD + q] = x[q];
                    P[r * SLD + c] = l;
                }
            } else {
                for (int r = c + 1 + t; r < m; r += 256) {
                    float l = P[r * SLD + c];
                    if (piv != 0.0f) l = l / piv;
                    P[r * SLD + c] = l;
                    for (int q = c + 1; q < jb; ++q) P[r * SLD + q] = fmaf(-l, P[c * SLD + q], P[r * SLD + q]);
                }
            }
            __syncthreads();
        }
        for (int e = t; e < m * SNB; e += 256) {
            const int r = e / SNB, q = e % SNB;
            if (q < jb) LU[(int64_t)(j + r) * n + j + q] = P[r * SLD + q];
        }
        // ---- the panel's interchanges on the other columns: composed into
        // one permutation of at most 2 jb rows (position d receives the old
        // row s), then every column's affected entries are all loaded before
        // any is stored
        __syncthreads();   // the panel's LDS is free
        {
            int *sp = reinterpret_cast<int *>(smem) + SWP_OFF;
            int *dpos = sp + SNB, *spos = dpos + 2 * SNB;
            int *s_nd = spos + 2 * SNB;
            if (t < jb) {
                const int q = it.ipiv[j + t] - j;   // >= t for a valid factorisation
                sp[t] = (q >= t && q < m) ? q : t;
            }
            if (t == 0) *s_nd = jb;
            __syncthreads();
            if (t < jb) {
                dpos[t] = t;
                const int q = sp[t];
                bool first = q >= jb;
                for (int k = 0; k < t && first; ++k) first = sp[k] != q;
                if (first) dpos[atomicAdd(s_nd, 1)] = q;
            }
            __syncthreads();
            const int nd = *s_nd;
            if (t < nd) {
                int pos = dpos[t];
                for (int i = jb - 1; i >= 0; --i) {
                    const int q = sp[i];
                    pos = (pos == i) ? q : ((pos == q) ? i : pos);
                }
                spos[t] = pos;
            }
            __syncthreads();
            float *tmp = reinterpret_cast<float *>(s_nd + 4);   // [2 SNB][256] staged entries
            // rows j .. n-1 of every column, addressed from row j
            const __amdgpu_buffer_rsrc_t rw = span_rsrc(LU + (int64_t)j * n, m * n);
            for (int col = t; col < n - jb; col += 256) {
                const int cc = col < j ? col : col + jb;
                // 16 loads in flight before their LDS stores
                for (int e0 = 0; e0 < nd; e0 += 16) {
                    float v[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int e = e0 + k;
                        v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                            rw, e < nd ? (spos[e < nd ? e : 0] * n + cc) * 4 : OOB, 0, 0));
                    }
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (e0 + k < nd) tmp[(e0 + k) * 256 + t] = v[k];
                }
                float *dst = LU + (int64_t)j * n + cc;
#pragma unroll 8
                for (int e = 0; e < nd; ++e) dst[(int64_t)dpos[e] * n] = tmp[e * 256 + t];
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
            {
                // the strictly lower part of L11: a thread's 4 loads in flight
                // before their LDS stores (other entries load as 0)
                const __amdgpu_buffer_rsrc_t rl = span_rsrc(LU + (int64_t)j * n + j, (jb - 1) * n + jb);
                float v[SNB * SNB / 256];
#pragma unroll
                for (int k = 0; k < SNB * SNB / 256; ++k) {
                    const int e = t + 256 * k, i = e / SNB, p = e % SNB;
                    v[k] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(rl, (i < jb && p < i) ? (i * n + p) * 4 : OOB, 0, 0));
                }
#pragma unroll
                for (int k = 0; k < SNB * SNB / 256; ++k) L[t + 256 * k] = v[k];
            }
            {
                // rows of A12: a thread's loads of 4 rows x 2 columns in
                // flight before their LDS stores
                const __amdgpu_buffer_rsrc_t rx = span_rsrc(LU + (int64_t)j * n + j + jb, (jb - 1) * n + rest);
                for (int i0 = 0; i0 < jb; i0 += 4)
                    for (int c0 = 0; c0 < rest; c0 += 512) {
                        float v[4][2];
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int i = i0 + ii, c = c0 + 256 * h + t;
                                v[ii][h] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                    rx, (i < jb && c < rest) ? (i * n + c) * 4 : OOB, 0, 0));
                            }
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int i = i0 + ii, c = c0 + 256 * h + t;
                                if (i < jb && c < rest) X[i * XLD + c] = v[ii][h];
                            }
                    }
            }
            __syncthreads();
            for (int c = t; c < rest; c += 256)
                for (int i = 1; i < jb; ++i) {
                    float s = X[i * XLD + c];
                    int p = 0;
                    // four terms' LDS reads issued together, then their FMAs
                    // in increasing p (the same chain as one term at a time)
                    for (; p + 4 <= i; p += 4) {
                        const float4 l4 = *reinterpret_cast<const float4 *>(L + i * SNB + p);
                        const float x0 = X[p * XLD + c], x1 = X[(p + 1) * XLD + c];
                        const float x2 = X[(p + 2) * XLD + c], x3 = X[(p + 3) * XLD + c];
                        s = fmaf(-l4.x, x0, s);
                        s = fmaf(-l4.y, x1, s);
                        s = fmaf(-l4.z, x2, s);
                        s = fmaf(-l4.w, x3, s);
                    }
                    for (; p < i; ++p) s = fmaf(-L[i * SNB + p], X[p * XLD + c], s);
                    X[i * XLD + c] = s;
                }
            __syncthreads();
            for (int i = 0; i < jb; ++i)
                for (int c = t; c < rest; c += 256) LU[(int64_t)(j + i) * n + j + jb + c] = X[i * XLD + c];
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
        if (jb == SNB) {
            rank32_update<V, true>(LU, n, j, rest);
        } else if (rest > 256) {
            // (a narrower last panel leaves no trailing matrix; kept general)
            const int tiles = (rest + 127) / 128;
            for (int tm = 0; tm < tiles; ++tm)
                for (int tn = 0; tn < tiles; ++tn)
                    gemm_tile<V, 128, 128, 2, 2>(gp, (int64_t)tm * 128, (int64_t)tn * 128, 0, jb, 0, smem);
        } else {
            const int tiles = (rest + 63) / 64;
            for (int tm = 0; tm < tiles; ++tm)
                for (int tn = 0; tn < tiles; ++tn)
                    gemm_tile<V, 64, 64, 2, 2>(gp, (int64_t)tm * 64, (int64_t)tn * 64, 0, jb, 0, smem);
        }
        __syncthreads();
    }

    // ---- iterative refinement (Sec. III)
    char *sb = reinterpret_cast<char *>(smem);
    float *y = reinterpret_cast<float *>(sb + L_Y);
    double *r = reinterpret_cast<double *>(sb + L_R);
    int32_t *perm = reinterpret_cast<int32_t *>(sb + L_PERM);
    float *D = reinterpret_cast<float *>(sb + L_D);
    const float *A = it.A;
    // norms
    double rowmax = 0.0;
    for (int row = wave; row < n; row += 4) {
        // the row's loads in flight together; each lane sums its entries in
        // increasing column order (elements past n load as 0 and are not added)
        const __amdgpu_buffer_rsrc_t ra = span_rsrc(A + (int64_t)row * it.lda, n);
        double s = 0.0;
        for (int c0 = 0; c0 < n; c0 += 512) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = c0 + lane + 64 * k;
                v[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ra, c < n ? c * 4 : OOB, 0, 0));
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + lane + 64 * k < n) s += fabs((double)v[k]);
        }
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
    block_trsv<float, true>(LU, n, y, D);
    block_trsv<float, false>(LU, n, y, D);
    for (int i = t; i < n; i += 256) it.x[i] = (double)y[i];
    __syncthreads();

    int iters = 0, rises = 0, status = 1, inner = 0;
    double eta = 0.0, prev_eta = INFINITY;
    for (; cfg.mode == 0;) {
        const double rn = residual_wg(it, n, r, reinterpret_cast<double *>(sb + L_V), s_d);
        const double xn = absmax_x_wg(it, n, s_d);
        const double den = normA * xn + normb;
        eta = den > 0.0 ? rn / den : rn;
        rises = (eta >= prev_eta) ? rises + 1 : 0;
        prev_eta = eta;
        status = ir_decide(eta, tol, iters, max_iter, rises);
        if (status >= 0) break;
        for (int i = t; i < n; i += 256) y[i] = (float)(r[perm[i]] / rn);
        __syncthreads();
        block_trsv<float, true>(LU, n, y, D);
        block_trsv<float, false>(LU, n, y, D);
        for (int i = t; i < n; i += 256) it.x[i] = fma(rn, (double)y[i], it.x[i]);
        __syncthreads();
        ++iters;
    }
    if (cfg.mode == 1 || ((status == 1 || status == 2) && cfg.max_iter > 0)) {
        if (cfg.mode == 0) {
            // LU-IR that stalls or diverges can leave x far worse than x0, and
            // GMRES-IR started there may stall as well: start it from x0.
            for (int i = t; i < n; i += 256) y[i] = (float)it.b[perm[i]];
            __syncthreads();
            block_trsv<float, true>(LU, n, y, D);
            block_trsv<float, false>(LU, n, y, D);
            for (int i = t; i < n; i += 256) it.x[i] = (double)y[i];
            __syncthreads();
        }
        status = gmres_phase(it, cfg, normA, normb, tol, smem, iters, inner, eta);
    }
    if (t == 0) {
        it.res->iters = iters;
        it.res->inner = inner;
        it.res->status = status;
        it.res->reserved = 0;
        it.res->eta = eta;
    }
    __syncthreads();
}

// Per-problem baseline results (bfx_ir_solve's) in the plan's result type.
__global__ void __launch_bounds__(64) ir_to_gmres_result(const bfx_ir_result *src, bfx_gmres_result *dst) {
    if (threadIdx.x == 0) {
        dst->iters = src->iters;
        dst->inner = 0;
        dst->status = src->status;
        dst->reserved = 0;
        dst->eta = src->eta;
    }
}

__global__ void __launch_bounds__(64) solve_zero_counter(uint32_t *c) {
    if (threadIdx.x == 0) *c = 0u;
}

template <int V>
__global__ void __launch_bounds__(256, 1)
persistent_solve_kernel(const SolveItem *__restrict__ items, int64_t count, uint32_t *counter,
                        double tol, int max_iter, GmresCfg cfg) {
    extern __shared__ __align__(16) uint16_t smem[];
    __shared__ int64_t s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t idx = s_idx;
        __syncthreads();
        if (idx >= count) break;
        solve_one<V>(items[idx], tol, max_iter, cfg, smem);
    }
}

}  // namespace bfx

struct bfx_solve_plan {
    int variant = 6;
    int64_t count = 0;
    bfx_batched_solve_opts opts = {1e-14, 30, 10, 0, 1e-8, 0, 0};
    std::vector<bfx_solve_desc> h_desc;
    std::vector<int64_t> lu_off, piv_off;   // host copies of per-problem offsets
    bfx::SolveItem *d_items = nullptr;
    float *d_lu = nullptr;
    int32_t *d_ipiv = nullptr;
    bfx_gmres_result *d_res = nullptr;
    bfx_ir_result *d_res_ir = nullptr;     // per-problem baseline
    int32_t *d_info = nullptr;
    double *d_scratch = nullptr;           // GMRES basis and Hessenberg, per workgroup
    int64_t m_cap = 0, per_wg = 0;
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
    if (p->d_res_ir) (void)hipFree(p->d_res_ir);
    if (p->d_info) (void)hipFree(p->d_info);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_ws) (void)hipFree(p->d_ws);
    delete p;
}
template <int V>
const void *solve_kernel_for() { return (const void *)persistent_solve_kernel<V>; }
}  // namespace
}  // namespace bfx

extern "C" int bfx_lu_ir_batched_plan_create(int variant, int64_t count, const bfx_solve_desc *descs,
                                             const bfx_batched_solve_opts *opts, bfx_solve_plan **out) {
    using namespace bfx;
    if (variant != 1 && variant != 3 && variant != 6 && variant != 9) return -1;
    if (count < 0) return -2;
    if (count > 0 && !descs) return -3;
    if (opts && (!(opts->tol >= 0.0) || opts->max_iter < 0 || opts->gmres_max_iter < 0 ||
                 opts->restart < 0 || !(opts->inner_tol >= 0.0) || opts->lu_format < 0 ||
                 opts->lu_format > 2 || opts->mode < 0 || opts->mode > 1 ||
                 (opts->mode == 1 && opts->gmres_max_iter == 0)))
        return -4;
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
    if ((e = hipMalloc(&p->d_res, sizeof(bfx_gmres_result) * cn)) != hipSuccess)
        return fail(e, "hipMalloc(plan results)");
    if ((e = hipMalloc(&p->d_res_ir, sizeof(bfx_ir_result) * cn)) != hipSuccess)
        return fail(e, "hipMalloc(plan baseline results)");
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
    if (p->opts.gmres_max_iter > 0 && count > 0) {
        // one slice per workgroup: basis (m_cap + 1) x nmax and R m_cap x m_cap
        int64_t nmax = 0;
        for (int64_t i = 0; i < count; ++i) nmax = std::max<int64_t>(nmax, descs[i].n);
        p->m_cap = p->opts.restart > 0 ? std::min<int64_t>(p->opts.restart, nmax) : nmax;
        p->per_wg = (p->m_cap + 1) * nmax + p->m_cap * p->m_cap;
        if ((e = hipMalloc(&p->d_scratch, sizeof(double) * p->per_wg * p->grid)) != hipSuccess)
            return fail(e, "hipMalloc(plan GMRES scratch)");
    }
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
        GmresCfg cfg;
        cfg.lu_format = p->opts.lu_format;
        cfg.mode = p->opts.mode;
        cfg.max_iter = p->d_scratch ? p->opts.gmres_max_iter : 0;
        cfg.restart = (int)p->m_cap;
        cfg.inner_tol = p->opts.inner_tol;
        cfg.m_cap = p->m_cap;
        cfg.scratch = p->d_scratch;
        cfg.per_wg = p->per_wg;
        void *args[] = {&p->d_items, &p->count, &p->d_counter, &tol, &max_iter, &cfg};
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
    if (p->opts.lu_format != 0 || p->opts.mode != 0) {
        set_error("bfx_solve_plan_launch_per_problem: only plans with the split-BF16 LU and LU-IR");
        return -1;
    }
    hipStream_t s = (hipStream_t)stream;
    for (int64_t i = 0; i < p->count; ++i) {
        const bfx_solve_desc &d = p->h_desc[i];
        float *lu = p->d_lu + p->lu_off[i];
        BFX_HIP(hipMemcpy2DAsync(lu, d.n * sizeof(float), d.A, d.lda * sizeof(float), d.n * sizeof(float),
                                 d.n, hipMemcpyDeviceToDevice, s));
        int rc = bfx_lu_factor(p->variant, d.n, lu, d.n, p->d_ipiv + p->piv_off[i], p->d_info + i, p->d_ws,
                               p->ws_bytes, s);
        if (rc) return rc;
        const bfx_ir_opts io = {p->opts.tol, p->opts.max_iter, 0};
        rc = bfx_ir_solve(d.n, d.A, d.lda, lu, d.n, p->d_ipiv + p->piv_off[i], d.b, d.x, &io,
                          p->d_res_ir + i, p->d_ws, p->ws_bytes, s);
        if (rc) return rc;
        hipLaunchKernelGGL(ir_to_gmres_result, dim3(1), dim3(64), 0, s, p->d_res_ir + i, p->d_res + i);
        BFX_LAUNCH_CHECK("per-problem result");
    }
    return BFX_OK;
}

extern "C" int bfx_solve_plan_results(const bfx_solve_plan *p, bfx_gmres_result *results, int32_t *info) {
    using namespace bfx;
    if (!p) return -1;
    BFX_HIP(hipDeviceSynchronize());
    if (results && p->count)
        BFX_HIP(hipMemcpy(results, p->d_res, sizeof(bfx_gmres_result) * p->count, hipMemcpyDeviceToHost));
    if (info && p->count)
        BFX_HIP(hipMemcpy(info, p->d_info, sizeof(int32_t) * p->count, hipMemcpyDeviceToHost));
    return BFX_OK;
}

extern "C" int bfx_solve_plan_factors(const bfx_solve_plan *p, int64_t index, float *lu, int32_t *ipiv) {
    using namespace bfx;
    if (!p) return -1;
    if (index < 0 || index >= p->count) return -2;
    BFX_HIP(hipDeviceSynchronize());
    const int64_t n = p->h_desc[index].n;
    if (lu) BFX_HIP(hipMemcpy(lu, p->d_lu + p->lu_off[index], sizeof(float) * n * n, hipMemcpyDeviceToHost));
    if (ipiv) BFX_HIP(hipMemcpy(ipiv, p->d_ipiv + p->piv_off[index], sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    return BFX_OK;
}

extern "C" int bfx_solve_plan_destroy(bfx_solve_plan *p) {
    if (!p) return -1;
    bfx::solve_plan_free(p);
    return BFX_OK;
}
