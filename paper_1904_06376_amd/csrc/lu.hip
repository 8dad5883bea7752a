// Blocked right-looking LU with partial pivoting (SGETRF semantics; the
// paper's split-BF16 LU, Sec. I and Sec. IV-A).  For every panel of up to 128
// columns:
//   1. panel_kernel  - FP32 factorisation of the (n-j) x jb panel.  The panel
//      rows are spread over G co-resident workgroups, 512 rows each, one row
//      per thread held in registers for the whole panel.  Per column every
//      workgroup publishes its best candidate row as words tagged with the
//      column, every workgroup reads all candidates in one round trip and
//      picks the same pivot (largest magnitude, lowest position on ties, as
//      ISAMAX); the previous column's elimination of a row runs while the
//      exchange is in flight, and interchanges move row labels.  The
//      candidate exchange is the only grid-wide synchronisation.  At the end
//      the panel writes its rows at their final positions and its
//      interchanges as a move list.
//   2. trsm_kernel   - for a range of trailing columns: the panel's
//      interchanges on those columns, then U12 = L11^{-1} A12 (unit lower,
//      FP32 FMA chains in index order, one wave per column).
//   3. laswp_kernel  - the interchanges on the columns left of the panel (and
//      on trailing columns whose trsm does not apply them).
//   4. A22 -= L21 x U12 with the split-BF16 GEMM (alpha = -1, beta = 1).
// With look-ahead (lu_lookahead) the next block column is updated first and
// its panel runs on its own compute units while the rest of the trailing
// matrix is updated; the serial schedule (lu_serial) runs 1-4 in order.
#include <climits>
#include <mutex>

#include <hip/hip_ext.h>

#include "common.hpp"

namespace bfx {

namespace {
constexpr int PNB = 128;     // panel width
constexpr int PROWS = 512;   // panel rows per workgroup (= threads, one row each in registers)
constexpr int MAX_G = 256;   // co-resident workgroups the panel may use
constexpr unsigned SPIN_LIMIT = 1u << 20;  // ~1 s of polling

// Column exchange words: {tag << 32 | 32-bit payload}, tag = global column
// index + 1, two slots per workgroup alternating with the column's parity.
// A slot holds the workgroup's candidate row: its register image as it was
// before the previous column's elimination (words 0..PNB-1), that
// elimination's multiplier (word PNB) and the row's position in the panel
// (word PNB + 1; -1: no candidate).
constexpr int CW = PNB + 4;      // words per slot
constexpr int XCH = PROWS / 16;  // candidates read per round (16 threads each)
constexpr int CRS = PNB + 4;     // LDS row stride of read candidates
// The panel's row interchanges as a move list for the rows outside it
// ([2][2 PNB] ints, by panel parity): entry q < w is the original panel
// position of the row that ends at position q; entry w + r (r < w) is the
// final position of original row r when that is >= w, else -1.
struct LuWs {
    uint64_t *cand;     // [2][MAX_G][CW] the workgroups' candidate rows
    int32_t *plan;      // [2][2 PNB] move lists
};

size_t lu_ws_layout(LuWs *w, void *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_cand = take(sizeof(uint64_t) * 2 * MAX_G * CW);
    const size_t o_plan = take(sizeof(int32_t) * 2 * 2 * PNB);
    if (w && base) {
        w->cand = (uint64_t *)((char *)base + o_cand);
        w->plan = (int32_t *)((char *)base + o_plan);
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


// Pivot keys: 0 for a row that takes no part (above the diagonal, or no row
// at all), else bits(|v|) + 1 with NaN taken as infinity (a NaN pivot wins and
// poisons the result).  Keys of non-negative floats order as the values; equal
// keys are broken by the lowest row, as ISAMAX does.
__device__ __forceinline__ uint32_t pivot_key(float v) {
    float av = fabsf(v);
    if (!(av == av)) av = INFINITY;
    return __float_as_uint(av) + 1u;
}

// Wave-wide maximum of a 32-bit key, returned uniform: DPP steps inside each
// row of 16 lanes (quad swaps, half-row and row mirrors), then the rows are
// chained by the row broadcasts so that lane 63 holds the maximum.  All 64
// lanes must be active.
__device__ __forceinline__ uint32_t wave_max_key(uint32_t x) {
    uint32_t y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x140, 0xF, 0xF, false);  // row_mirror
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    x = x > y ? x : y;
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Wave-wide minimum of a 32-bit value, returned uniform (the same DPP steps).
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    uint32_t y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0xB1, 0xF, 0xF, false);
    x = x < y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x4E, 0xF, 0xF, false);
    x = x < y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x141, 0xF, 0xF, false);
    x = x < y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x140, 0xF, 0xF, false);
    x = x < y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x142, 0xA, 0xF, false);
    x = x < y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x143, 0xC, 0xF, false);
    x = x < y ? x : y;
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// The lane holding the largest key, the lowest position among equal keys:
// returns that lane (uniform) and the maximum key in m.  Lanes whose key
// is 0 take no part (m = 0 then).
__device__ __forceinline__ int best_lane(uint32_t key, uint32_t pos, uint32_t &m) {
    m = wave_max_key(key);
    const uint64_t ties = __ballot(key == m);
    if (__popcll(ties) == 1) return __builtin_ctzll(ties);
    const uint32_t pm = wave_min_u32(key == m ? pos : 0xffffffffu);
    return __builtin_ctzll(__ballot(key == m && pos == pm));
}

// lowest lane whose predicate holds (64 if none)
__device__ __forceinline__ int first_lane(bool pred) {
    const uint64_t b = __ballot(pred);
    return b ? __builtin_ctzll(b) : 64;
}

// Bounded wait until every word of a tagged exchange read carries the tag:
// returns false (and records info = -1) when the wait expires or another
// workgroup's wait already did.
__device__ __forceinline__ bool wait_expired(unsigned &spins, int32_t *info) {
    if (++spins > SPIN_LIMIT ||
        ((spins & 255u) == 0 && __hip_atomic_load(info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == -1)) {
        __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    __builtin_amdgcn_s_sleep(2);
    return false;
}

// Each thread holds one panel row in registers, r[0..PNB-1], in a layout
// that keeps the current column in r[0]: after k eliminations (k = the
// column index for rows still below the diagonal) r[0 .. w-k-1] hold columns
// k .. w-1, r[PNB-k .. PNB-1] hold the multipliers l_0 .. l_{k-1}, and the
// registers between are padding.  An elimination shifts the row left by one
// (r[i] = r[i+1] - l U[i+1] on the live part, a plain shift elsewhere) and
// puts the new multiplier in r[PNB-1]; all register indices are static.  Rows
// that reach the diagonal freeze.
//
// Interchanges move labels, not data: each thread carries the position of
// the row it holds (pos).  When row p is chosen as pivot of column c, the
// thread holding it takes position c and freezes, and the thread holding
// position c takes position p; both images were shifted c times, so each
// thread's registers are exactly the row at its new position.  Rows go to
// their final positions at the write-back.  Ties between equal pivot
// magnitudes go to the lowest position, as ISAMAX.
//
// The elimination of column c-1 is deferred past the pivot search of column
// c: once pivot c-1 is known, every row computes its multiplier and only its
// next column entry (one FMA), which gives the pivot keys of column c.  The
// workgroup's candidate is published as it was before that elimination,
// with its multiplier, and every reader applies the elimination itself while
// storing it (the same FMA, so the same bits); the owner's full-row update
// runs while the exchange is in flight.
//
// Per column, two workgroup barriers.  Before the first, every wave has its
// best pivot key (DPP maximum) and that row's position in LDS; after it every
// wave forms the workgroup's candidate from the eight wave maxima and the
// wave holding it publishes it as words tagged with the column (a reader
// that sees the column's tag in a word has that word's value, so no fence
// orders the stores).  Every thread then reads its share of all candidates
// (16 threads per candidate, one 128-byte segment per load instruction and
// candidate), polling its own words.  After the second barrier every wave
// picks the same pivot.
__global__ void __launch_bounds__(PROWS, 1) panel_kernel(PanelArgs a) {
    // the workgroup's candidate staged for publishing (image, multiplier)
    __shared__ __align__(16) float rowbuf[PNB + 4];
    // candidate rows read from the exchange (after the elimination), element
    // q of candidate k at crow[.][k][3 + q], so that elements 1, 5, 9, ...
    // start 16-byte groups; two buffers alternate with the column, since
    // the readers of column c apply the elimination by pivot row c-1.  ubuf
    // holds the best row of earlier rounds when there are several.
    __shared__ __align__(16) float crow[2][XCH][CRS];
    __shared__ __align__(16) float ubuf[2][CRS];
    __shared__ int cidx[XCH];
    __shared__ uint32_t red_key[PROWS / 64], red_pos[PROWS / 64];
    __shared__ int red_lane[PROWS / 64];

    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w = a.w;
    const int row0 = g * PROWS;                    // first panel row of this workgroup
    const bool own = row0 + t < a.m;               // this thread holds a row
    int pos = row0 + t;                            // position of the row it holds
    float *Ag = a.A + a.j * a.lda + a.j;           // panel origin
    float r[PNB];
#pragma unroll
    for (int k = 0; k < PNB; ++k) r[k] = (own && k < w) ? Ag[(int64_t)pos * a.lda + k] : 0.0f;
    float l = 0.0f;   // this row's multiplier of the deferred elimination

    // the elimination of one column on this thread's row: multiplier l,
    // pivot row U1[k] = U[k + 1], live = width of that column's live part
    auto eliminate = [&](const float *U1, int live) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < PNB / 8; ++b) {
            if (8 * b + 8 <= live - 1) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = 8 * b + i;
                    if (k < PNB - 1) r[k] = fmaf(-l, U1[k], r[k + 1]);
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
                    if (k < PNB - 1) r[k] = (k < live - 1) ? fmaf(-l, U1[k], r[k + 1]) : r[k + 1];
                }
            }
        }
        r[PNB - 1] = l;
    };
    // pivot keys of column c from the entries v; this wave's best to LDS
    auto wave_keys = [&](int c, float v) __attribute__((always_inline)) {
        const uint32_t key = (own && pos >= c) ? pivot_key(v) : 0u;
        uint32_t m;
        const int lw = best_lane(key, (uint32_t)pos, m);
        if (lane == 0) {
            red_key[wave] = m;
            red_pos[wave] = (uint32_t)__builtin_amdgcn_readlane(pos, lw);
            red_lane[wave] = lw;
        }
    };

    wave_keys(0, r[0]);
    const float *Up = nullptr;   // pivot row of the previous column (LDS), U[k] at Up[3 + k]
    for (int c = 0; c < w; ++c) {
        const int par = c & 1;
        const uint32_t tag = (uint32_t)(a.j + c + 1);   // never 0 (exchange words start zeroed)
        const int live_p = w - c + 1;   // live width of the deferred elimination (column c-1)
        __syncthreads();
        // ---- the workgroup's candidate: the best of the wave maxima
        {
            const bool lw8 = lane < PROWS / 64;
            const uint32_t wk = lw8 ? red_key[lane] : 0u;
            const uint32_t wp = lw8 ? red_pos[lane] : 0xffffffffu;
            uint32_t M;
            const int W = best_lane(wk, wp, M);
            const int Wc = W < PROWS / 64 ? W : 0;
            const int L = red_lane[Wc];
            const int cand = M ? (int)red_pos[Wc] : -1;
            if (wave == (M ? Wc : 0)) {
                if (M && lane == L) {
#pragma unroll
                    for (int k = 0; k < PNB; ++k) rowbuf[k] = r[k];
                    rowbuf[PNB] = l;
                }
                const uint64_t tg = (uint64_t)tag << 32;
                uint64_t *slot = a.ws.cand + (size_t)(par * MAX_G + g) * CW;
                __hip_atomic_store(slot + lane, tg | __float_as_uint(rowbuf[lane]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(slot + lane + 64, tg | __float_as_uint(rowbuf[lane + 64]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                if (lane == 0) {
                    __hip_atomic_store(slot + PNB, tg | __float_as_uint(rowbuf[PNB]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(slot + PNB + 1, tg | (uint32_t)cand, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        // ---- the deferred elimination of column c-1 on this thread's row
        if (c > 0 && own && pos >= c) eliminate(Up + 4, live_p);
        // ---- read every candidate, eliminating column c-1 on the way (word
        // q + 1 of the slot gives element q; the last element is the
        // multiplier itself); then pick the pivot
        uint32_t best = 0;
        int bidx = -1;
        const float *Uc = crow[par][0];
        const int o = c > 0 ? 1 : 0;
        for (int k0 = 0; k0 < a.G; k0 += XCH) {
            const int kl = t >> 4, sub = t & 15;
            if (k0 + kl < a.G) {
                const uint64_t *src = a.ws.cand + (size_t)(par * MAX_G + k0 + kl) * CW;
                uint64_t wv[8], wl = 0, wi = 0;
                for (unsigned spins = 0;;) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        wv[q] = __hip_atomic_load(src + sub + o + 16 * q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    wl = __hip_atomic_load(src + PNB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    bool ok = (uint32_t)(wl >> 32) == tag;
                    if (sub == 0) {
                        wi = __hip_atomic_load(src + PNB + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = ok && (uint32_t)(wi >> 32) == tag;
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) ok = ok && (uint32_t)(wv[q] >> 32) == tag;
                    if (ok || wait_expired(spins, a.info)) break;
                }
                const float lk = __uint_as_float((uint32_t)wl);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int e = sub + 16 * q;
                    float x = __uint_as_float((uint32_t)wv[q]);
                    if (c > 0 && e < live_p - 1) x = fmaf(-lk, Up[4 + e], x);
                    crow[par][kl][3 + e] = x;
                }
                if (sub == 0) cidx[kl] = (int)(uint32_t)wi;
            }
            __syncthreads();
            // every wave: the best candidate of this round, kept if it beats
            // earlier rounds (which hold lower positions on equal keys)
            uint32_t key = 0, cp = 0xffffffffu;
            if (lane < XCH && k0 + lane < a.G && cidx[lane] >= 0) {
                key = pivot_key(crow[par][lane][3]);
                cp = (uint32_t)cidx[lane];
            }
            uint32_t m;
            const int kw = best_lane(key, cp, m);
            const int kwc = kw < XCH ? kw : 0;
            if (a.G <= XCH) {
                best = m;
                bidx = m ? cidx[kwc] : -1;
                Uc = crow[par][kwc];
            } else {
                const bool better = k0 == 0 || m > best || (m == best && m && cidx[kwc] < bidx);
                if (better) {
                    best = m;
                    bidx = m ? cidx[kwc] : -1;
                    if (t < PNB) ubuf[par][3 + t] = crow[par][kwc][3 + t];
                }
                Uc = ubuf[par];
                __syncthreads();   // ubuf complete; crow free for the next round
            }
        }
        // a valid pivot position is >= c; anything else only follows an expired wait
        const int p = (bidx >= c && bidx < a.m) ? bidx : c;
        const float piv = Uc[3];
        if (g == 0 && t == 0) {
            a.ipiv[a.j + c] = (int32_t)(a.j + p);
            if (piv == 0.0f && *a.info == 0) *a.info = (int32_t)(a.j + c + 1);  // -1 (expired wait) is kept
        }
        // ---- interchange positions c and p (labels); the multipliers of
        // the rows below and their entries in column c+1 (the rest of the
        // elimination is deferred)
        float v1 = 0.0f;
        if (own && pos >= c) {
            if (pos == p) pos = c;
            else if (pos == c) pos = p;
            if (pos > c) {
                l = r[0];
                if (piv != 0.0f) l = l / piv;
                v1 = (w - c > 1) ? fmaf(-l, Uc[4], r[1]) : r[1];
            }
        }
        Up = Uc;
        if (c + 1 < w) wave_keys(c + 1, v1);
    }
    // the last column's elimination
    if (own && pos >= w) eliminate(Up + 4, 1);

    // ---- the move list for the columns outside the panel (a thread's
    // original position is row0 + t, its final one pos)
    if (own) {
        int32_t *plan = a.ws.plan + ((a.j / PNB) & 1) * 2 * PNB;
        if (pos < w) plan[pos] = row0 + t;
        if (row0 + t < w) plan[w + row0 + t] = pos >= w ? pos : -1;
    }
    // ---- write back to the row's final position: register k of a row
    // shifted s times holds column s + k (k < w - s) or multiplier
    // k - (PNB - s) (k >= PNB - s)
    if (own) {
        const int sh = (pos < w) ? pos : w;
        float *Ar = Ag + (int64_t)pos * a.lda;
#pragma unroll
        for (int k = 0; k < PNB; ++k) {
            int col = -1;
            if (k < w - sh) col = sh + k;
            else if (k >= PNB - sh) col = k - (PNB - sh);
            if (col >= 0) Ar[col] = r[k];
        }
    }
}

__global__ void __launch_bounds__(256) zero_u64(uint64_t *p, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0ull;
}

// Row interchanges of rows j..j+w-1 (ipiv, applied in order, LAPACK laswp
// semantics) on columns outside the panel, from the panel's move list: the
// affected positions are the panel rows 0..w-1 and the rows beyond them that
// received a panel row.  Every thread of the workgroup calls this; on return
// dpos[0..nd) are the affected positions and spos[e] is the position whose
// old row moves to dpos[e].
constexpr int SWP_MAXR = 2 * PNB;  // affected rows: the panel rows and at most w others
__device__ int read_moves(const int32_t *plan, int w, int *dpos, int *spos, int *s_nd) {
    const int t = threadIdx.x;
    if (t == 0) *s_nd = w;
    __syncthreads();
    if (t < w) {
        dpos[t] = t;
        spos[t] = plan[t];
        const int q = plan[w + t];
        if (q >= w) {
            const int e = atomicAdd(s_nd, 1);
            dpos[e] = q;
            spos[e] = t;
        }
    }
    __syncthreads();
    return *s_nd;
}

// The panel's interchanges on the columns [0, x1) and [x2, n).  Every
// affected row of the workgroup's 64 columns is loaded (coalesced 256-byte
// row segments, many loads in flight), all loads complete before the
// barrier, and the rows are stored at their new positions.
constexpr int SWP_COLS = 64;       // columns per workgroup
constexpr int SWP_THREADS = 256;   // 4 waves: wave v moves affected rows v, v+4, ...
__global__ void __launch_bounds__(SWP_THREADS)
laswp_kernel(float *A, int64_t lda, int64_t n, int64_t j, int w, const int32_t *plan, int64_t x1, int64_t x2) {
    __shared__ int dpos[SWP_MAXR], spos[SWP_MAXR];
    __shared__ int s_nd;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int nd = read_moves(plan, w, dpos, spos, &s_nd);
    int64_t col = (int64_t)blockIdx.x * SWP_COLS + lane;
    if (col >= x1) col += x2 - x1;
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

// U12 = L11^{-1} A12 (unit lower L11, jb x jb), with the panel's row
// interchanges applied to the same columns first.  The interchanges: every
// affected row of the workgroup's columns is loaded (16-column row segments),
// all loads complete before the barrier, then rows beyond the panel are
// stored at their new positions and the panel rows go to LDS as the
// right-hand sides.  The solve is the column-oriented forward substitution:
// at step p the now final x_p is broadcast and every row i > p is updated,
// x_i = fma(-L_ip, x_p, x_i) -- for each element the same FMA chain, in
// increasing p, as the row-oriented algorithm.  One wave per column, lane l
// holding rows l and l + 64: x_p is read from its lane (readlane) as soon as
// the previous step has made it final, so the solve has no barrier.  A
// 1024-thread workgroup owns 16 columns; L11 is staged transposed in LDS
// (rows padded to 129 floats: conflict-free both ways).
constexpr int TRSM_COLS = 16;
constexpr int TRSM_LD = PNB + 1;
constexpr size_t TRSM_LDS = (size_t)(PNB + TRSM_COLS) * TRSM_LD * sizeof(float);
__global__ void __launch_bounds__(1024)
trsm_kernel(float *A, int64_t lda, int64_t n, int64_t c0, int64_t c1, int64_t j, int w, const int32_t *plan) {
    extern __shared__ float tsm[];
    float *Lt = tsm;                    // Lt[p * TRSM_LD + i] = L11[i][p] for p < i < w, else 0
    float *Xs = tsm + PNB * TRSM_LD;    // Xs[c * TRSM_LD + i] = A12[i][c]
    __shared__ int dpos[SWP_MAXR], spos[SWP_MAXR];
    __shared__ int s_nd;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int64_t cb = c0 + (int64_t)blockIdx.x * TRSM_COLS;   // columns [c0, c1)
    // plan == nullptr: the interchanges were applied already
    const int nd = plan ? read_moves(plan, w, dpos, spos, &s_nd) : 0;
    // the interchanges: thread t moves column t % 16 of affected rows
    // t / 16, t / 16 + 64, ...
    const int sc = t & (TRSM_COLS - 1), se = t / TRSM_COLS;
    const bool cok = cb + sc < c1;
    constexpr int SPER = SWP_MAXR / (1024 / TRSM_COLS);
    float v[SPER];
#pragma unroll
    for (int k = 0; k < SPER; ++k) {
        const int e = se + (1024 / TRSM_COLS) * k;
        v[k] = (cok && e < nd) ? A[(j + spos[e]) * lda + cb + sc] : 0.0f;
    }
    if ((int64_t)PNB * lda * 4 >= (int64_t(1) << 31)) {
        // rows too far apart for 32-bit buffer offsets
        for (int e = t; e < PNB * PNB; e += 1024) {
            const int i = e / PNB, p = e % PNB;
            Lt[p * TRSM_LD + i] = (i < w && p < i) ? A[(j + i) * lda + j + p] : 0.0f;
        }
    } else {
        // L11: a thread's 16 loads in flight before their LDS stores (entries
        // on or above the diagonal take an out-of-range offset and load as 0)
        const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(A + j * lda + j), (short)0, (int)(((w - 1) * lda + w) * 4), 0x00020000);
        float lv[PNB * PNB / 1024];
#pragma unroll
        for (int k = 0; k < PNB * PNB / 1024; ++k) {
            const int e = t + 1024 * k, i = e / PNB, p = e % PNB;
            lv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                rl, (i < w && p < i) ? (int)((i * lda + p) * 4) : 0x40000000, 0, 0));
        }
#pragma unroll
        for (int k = 0; k < PNB * PNB / 1024; ++k) {
            const int e = t + 1024 * k, i = e / PNB, p = e % PNB;
            Lt[p * TRSM_LD + i] = lv[k];
        }
    }
    if (!plan) {
        for (int e = t; e < PNB * TRSM_COLS; e += 1024) {
            const int i = e / TRSM_COLS, c = e % TRSM_COLS;
            Xs[c * TRSM_LD + i] = (i < w && cb + c < c1) ? A[(j + i) * lda + cb + c] : 0.0f;
        }
    } else {
        for (int e = t; e < PNB * TRSM_COLS; e += 1024) Xs[(e / PNB) * TRSM_LD + e % PNB] = 0.0f;
    }
    // every load of the workgroup has returned before any row is overwritten
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SPER; ++k) {
        const int e = se + (1024 / TRSM_COLS) * k;
        if (e < nd) {
            const int q = dpos[e];
            if (q < w) Xs[sc * TRSM_LD + q] = v[k];
            else if (cok) A[(j + q) * lda + cb + sc] = v[k];
        }
    }
    __syncthreads();
    float x0 = Xs[wv * TRSM_LD + lane], x1 = Xs[wv * TRSM_LD + lane + 64];
    // all PNB - 1 steps, branch-free: rows at or beyond w are zero padding
    // (never stored), so the steps past w - 1 change no stored row
#pragma unroll
    for (int p0 = 0; p0 < 64; p0 += 8) {            // x_p in lane p's x0
        float la[8], lb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            la[q] = Lt[(p0 + q) * TRSM_LD + lane];
            lb[q] = Lt[(p0 + q) * TRSM_LD + lane + 64];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = p0 + q;
            const float xp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x0), p));
            const float y0 = fmaf(-la[q], xp, x0);
            x0 = (lane > p) ? y0 : x0;
            x1 = fmaf(-lb[q], xp, x1);              // rows lane + 64 > p
        }
    }
#pragma unroll
    for (int p0 = 64; p0 < PNB; p0 += 8) {          // x_p in lane p-64's x1
        float lb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) lb[q] = Lt[(p0 + q) * TRSM_LD + lane + 64];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = p0 + q;
            if (p == PNB - 1) break;
            const float xp = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x1), p - 64));
            const float y1 = fmaf(-lb[q], xp, x1);
            x1 = (lane + 64 > p) ? y1 : x1;
        }
    }
    Xs[wv * TRSM_LD + lane] = x0;
    Xs[wv * TRSM_LD + lane + 64] = x1;
    __syncthreads();
    for (int e = t; e < PNB * TRSM_COLS; e += 1024) {
        const int i = e / TRSM_COLS, c = e % TRSM_COLS;
        if (i < w && cb + c < c1) A[(j + i) * lda + cb + c] = Xs[c * TRSM_LD + i];
    }
}

static int set_trsm_attr() {
    static bool attr = false;
    if (!attr) {
        BFX_HIP(hipFuncSetAttribute((const void *)trsm_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)TRSM_LDS));
        attr = true;
    }
    return BFX_OK;
}

// U12 = L11^{-1} A12 and A22 -= L21 U12 for the columns [c0, c1) of the
// trailing matrix of the panel at j (rows j + jb .. n-1); with the panel's
// move list, its interchanges on those columns first (else they were applied).
static int lu_update_cols(int variant, int64_t n, float *A, int64_t lda, const int32_t *plan, int64_t j, int jb,
                          int64_t c0, int64_t c1, hipStream_t s, int cus) {
    if (c1 <= c0) return BFX_OK;
    hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)ceil_div(c1 - c0, TRSM_COLS)), dim3(1024), TRSM_LDS, s,
                       A, lda, n, c0, c1, j, jb, plan);
    BFX_LAUNCH_CHECK("trsm_kernel");
    const int64_t rows = n - j - jb;
    if (rows <= 0) return BFX_OK;
    const float *A21 = A + (j + jb) * lda + j;
    const float *A12 = A + j * lda + c0;
    float *A22 = A + (j + jb) * lda + c0;
    // variant 0: the plain FP32 vector GEMM (an SGETRF built on SGEMM, the
    // comparator of Sec. IV-A's LU experiment)
    return variant == 0 ? bfx_sgemm_fp32(rows, c1 - c0, jb, -1.0f, A21, lda, A12, lda, 1.0f, A22, lda, nullptr, 0,
                                         (void *)s)
                        : gemm_launch(variant, rows, c1 - c0, jb, -1.0f, A21, lda, A12, lda, 1.0f, A22, lda,
                                      nullptr, 0, s, 0, cus);
}

static PanelArgs panel_args(float *A, int64_t lda, int64_t n, int64_t j, int32_t *ipiv, int32_t *info,
                            const LuWs &w) {
    PanelArgs pa;
    pa.A = A; pa.lda = lda; pa.n = n; pa.j = j; pa.m = n - j;
    pa.w = (int)((n - j < PNB) ? n - j : PNB);
    pa.G = (int)ceil_div(n - j, PROWS);
    pa.ipiv = ipiv; pa.info = info; pa.ws = w;
    return pa;
}

static const int32_t *plan_of(const LuWs &w, int64_t j) { return w.plan + ((j / PNB) & 1) * 2 * PNB; }

// the panel's interchanges on the columns [0, x1) and [x2, n)
static int launch_laswp(float *A, int64_t lda, int64_t n, int64_t j, int jb, const int32_t *plan, int64_t x1,
                        int64_t x2, hipStream_t s) {
    const int64_t cols = x1 + (n - x2);
    if (cols <= 0) return BFX_OK;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)ceil_div(cols, SWP_COLS)), dim3(SWP_THREADS), 0, s, A, lda,
                       n, j, jb, plan, x1, x2);
    BFX_LAUNCH_CHECK("laswp_kernel");
    return BFX_OK;
}

// One stream: panel (cooperative launch over the whole device), row
// interchanges, U12, trailing update, in order.
static int lu_serial(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv, int32_t *info,
                     const LuWs &w, hipStream_t s) {
    for (int64_t j = 0; j < n; j += PNB) {
        PanelArgs pa = panel_args(A, lda, n, j, ipiv, info, w);
        void *args[] = {&pa};
        BFX_HIP(hipLaunchCooperativeKernel((const void *)panel_kernel, dim3(pa.G), dim3(PROWS), args, 0, s));
        int rc = launch_laswp(A, lda, n, j, pa.w, plan_of(w, j), j, j + pa.w, s);
        if (rc != BFX_OK) return rc;
        rc = lu_update_cols(variant, n, A, lda, nullptr, j, pa.w, j + pa.w, n, s, 0);
        if (rc != BFX_OK) return rc;
    }
    return BFX_OK;
}

// Depth-1 look-ahead over two CU-masked streams: the panel stream runs on
// PANEL_CUS compute units (the first PANEL_CUS bits of the mask, which the
// driver spreads evenly over the XCDs), the update stream on all the others.
// After panel k, the update stream applies its interchanges, then updates the
// next block column first; the panel stream factors that column (panel k+1)
// while the update stream updates the rest of the trailing matrix.  The
// arithmetic and its order are those of the serial schedule (each trailing
// element sees the same updates in the same order), so the factors are the
// same bits.  The panel launch is a plain one: its G <= PANEL_CUS workgroups
// each fill a compute unit and nothing else runs on those units, so all of
// them are resident together.  A panel too tall for PANEL_CUS units runs on
// the update stream, in order.  Streams and events are created once per
// device and kept for the life of the process; one mutex per device orders
// concurrent callers' launch sequences.
constexpr int PANEL_CUS = 32;
struct LuStreams {
    bool tried = false, ok = false;
    hipStream_t sp = nullptr, sg = nullptr;
    hipEvent_t e0 = nullptr, en = nullptr, ep = nullptr, ef = nullptr;
    int update_cus = 0;
    std::mutex mu;
};
static LuStreams g_lu_streams[64];
static std::mutex g_lu_streams_mu;

static LuStreams *lu_streams() {
    const char *off = getenv("BFX_LU_LOOKAHEAD");   // "0": the serial schedule
    if (off && off[0] == '0') return nullptr;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    LuStreams &L = g_lu_streams[dev];
    std::lock_guard<std::mutex> lock(g_lu_streams_mu);
    if (!L.tried) {
        L.tried = true;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 2 * PANEL_CUS || cus > 1024)
            return nullptr;
        uint32_t mp[32] = {0}, mg[32] = {0};
        const int words = (cus + 31) / 32;
        for (int c = 0; c < cus; ++c) {
            if (c < PANEL_CUS) mp[c / 32] |= 1u << (c % 32);
            else mg[c / 32] |= 1u << (c % 32);
        }
        bool ok = hipExtStreamCreateWithCUMask(&L.sp, words, mp) == hipSuccess &&
                  hipExtStreamCreateWithCUMask(&L.sg, words, mg) == hipSuccess;
        for (hipEvent_t *e : {&L.e0, &L.en, &L.ep, &L.ef})
            ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
        (void)hipGetLastError();
        L.update_cus = cus - PANEL_CUS;
        L.ok = ok;
    }
    return L.ok ? &L : nullptr;
}

static int lu_lookahead(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv, int32_t *info,
                        const LuWs &w, hipStream_t s, LuStreams &L) {
    std::lock_guard<std::mutex> lock(L.mu);
    hipStream_t sp = L.sp, sg = L.sg;
    const int ucus = L.update_cus;
    // both streams start after the work already queued on s
    BFX_HIP(hipEventRecord(L.e0, s));
    BFX_HIP(hipStreamWaitEvent(sp, L.e0, 0));
    BFX_HIP(hipStreamWaitEvent(sg, L.e0, 0));
    // panel at j: on the panel stream when it fits there (its event ep is
    // recorded; the caller queues the update stream's wait for it), else on
    // the update stream
    auto panel_small = [&](int64_t j) { return ceil_div(n - j, PROWS) <= PANEL_CUS; };
    auto launch_panel = [&](int64_t j) -> int {
        PanelArgs pa = panel_args(A, lda, n, j, ipiv, info, w);
        hipStream_t ps = sp;
        if (pa.G > PANEL_CUS) {
            if (pa.G > ucus) return -2;
            ps = sg;
        }
        hipLaunchKernelGGL(panel_kernel, dim3(pa.G), dim3(PROWS), 0, ps, pa);
        BFX_LAUNCH_CHECK("panel_kernel");
        if (ps == sp) BFX_HIP(hipEventRecord(L.ep, sp));
        return BFX_OK;
    };
    int rc = launch_panel(0);
    if (rc == BFX_OK && panel_small(0)) BFX_HIP(hipStreamWaitEvent(sg, L.ep, 0));
    for (int64_t j = 0; j < n && rc == BFX_OK; j += PNB) {
        const int jb = (int)((n - j < PNB) ? n - j : PNB);
        const int64_t c0 = j + jb;
        const int32_t *plan = plan_of(w, j);
        if (c0 >= n) {
            rc = launch_laswp(A, lda, n, j, jb, plan, j, n, sg);
            break;
        }
        const int64_t c1 = (n - c0 < PNB) ? n : c0 + PNB;
        // the next block column first (its interchanges in the same kernel)
        rc = lu_update_cols(variant, n, A, lda, plan, j, jb, c0, c1, sg, ucus);
        if (rc != BFX_OK) break;
        const bool small = panel_small(c0);
        if (small) {
            // its panel on the panel stream, beside the rest of the update
            BFX_HIP(hipEventRecord(L.en, sg));
            BFX_HIP(hipStreamWaitEvent(sp, L.en, 0));
            rc = launch_panel(c0);
            if (rc != BFX_OK) break;
        }
        // the interchanges left of the panel and right of the next block
        // column, then the rest of the trailing update
        rc = launch_laswp(A, lda, n, j, jb, plan, j, c1, sg);
        if (rc != BFX_OK) break;
        rc = lu_update_cols(variant, n, A, lda, nullptr, j, jb, c1, n, sg, ucus);
        if (rc != BFX_OK) break;
        if (small) BFX_HIP(hipStreamWaitEvent(sg, L.ep, 0));
        else rc = launch_panel(c0);
    }
    if (rc != BFX_OK) return rc;
    BFX_HIP(hipEventRecord(L.ef, sp));
    BFX_HIP(hipStreamWaitEvent(s, L.ef, 0));
    BFX_HIP(hipEventRecord(L.ef, sg));
    BFX_HIP(hipStreamWaitEvent(s, L.ef, 0));
    return BFX_OK;
}

static int lu_factor_impl(int variant, int64_t n, float *A, int64_t lda, int32_t *ipiv,
                          int32_t *info, void *ws, hipStream_t s) {
    LuWs w;
    lu_ws_layout(&w, ws);
    int rc = set_trsm_attr();
    if (rc != BFX_OK) return rc;
    BFX_HIP(hipMemsetAsync(info, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(zero_u64, dim3(64), dim3(256), 0, s, w.cand, 2 * MAX_G * CW);
    BFX_LAUNCH_CHECK("zero_u64");
    if (LuStreams *L = lu_streams()) return lu_lookahead(variant, n, A, lda, ipiv, info, w, s, *L);
    return lu_serial(variant, n, A, lda, ipiv, info, w, s);
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
