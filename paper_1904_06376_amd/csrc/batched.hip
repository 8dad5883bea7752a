// Many independent split-BF16 GEMMs in one persistent, graph-captured launch.
//
// plan_create: validates the descriptors, picks a tile shape per problem from
// the tuning table (by M/N bucket; built-in default otherwise), expands every
// problem into output tiles, orders the tiles by estimated cost, longest first
// (LPT), and uploads descriptors and the tile list.  plan_launch: on first use
// captures "reset the work counter + one persistent kernel" into a HIP graph,
// then replays the graph on the caller's stream.  The persistent kernel keeps
// one workgroup per resident slot; each takes the next tile index with an
// atomic add and runs the shared tile engine until the list is exhausted, so
// every workgroup reaches the exit.  Problems the wave-specialised engine can
// take (K % 4 == 0, 16-byte aligned A rows) go to one persistent kernel of
// 512-thread workgroups, the others to one of 256-thread workgroups running
// the general engine; both kernels sit in the same graph, one after the other.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gemm_tile.hpp"

namespace bfx {

namespace {
// 0-3: general engine tiles; 4-5: wave-specialised tiles.
enum { CFG_64x64 = 0, CFG_128x128 = 1, CFG_128x64 = 2, CFG_64x128 = 3, CFG_F64 = 4, CFG_F128 = 5,
       NCFG = 6 };
const int cfg_bm[NCFG] = {64, 128, 128, 64, 64, 128};
const int cfg_bn[NCFG] = {64, 128, 64, 128, 64, 128};
bool cfg_fast(int c) { return c >= CFG_F64; }

struct TileItem {
    int32_t prob, tm, tn, cfg;
};

int bucket(int64_t x) { return x <= 64 ? 0 : x <= 128 ? 1 : x <= 256 ? 2 : 3; }
}  // namespace

__global__ void __launch_bounds__(64) plan_zero_counter(uint32_t *c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

__device__ __forceinline__ GemmParams desc_params(const bfx_gemm_desc &d) {
    GemmParams p;
    p.M = d.M; p.N = d.N; p.K = d.K;
    p.A = d.A; p.lda = d.lda; p.B = d.B; p.ldb = d.ldb; p.C = d.C; p.ldc = d.ldc;
    p.alpha = d.alpha; p.beta = d.beta;
    p.k_per_split = d.K; p.splits = 1; p.partial = nullptr;
    p.vecA = ((uintptr_t)d.A % 16 == 0) && (d.lda % 4 == 0);
    p.vecB = ((uintptr_t)d.B % 16 == 0) && (d.ldb % 4 == 0);
    return p;
}

// Wave-specialised persistent kernel (512 threads).  WIDE = false: only the
// 64 x 64 tile (half the LDS, two workgroups per CU); true: 64 and 128.
template <int V, bool WIDE>
__global__ void __launch_bounds__(512, WIDE ? 1 : 2)
persistent_fast_kernel(const bfx_gemm_desc *__restrict__ probs,
                       const TileItem *__restrict__ tiles, int64_t ntiles, uint32_t *counter) {
    extern __shared__ __align__(16) uint16_t smem[];
    __shared__ int64_t s_idx;
    for (;;) {
        // taken by a helper-wave thread: the MFMA waves may still have C
        // stores in flight, which a wait for the atomic's return would
        // also wait for
        if (threadIdx.x == 256) s_idx = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t idx = s_idx;
        __syncthreads();
        if (idx >= ntiles) break;
        const TileItem t = tiles[idx];
        const bfx_gemm_desc d = probs[t.prob];
        const GemmParams p = desc_params(d);
        if (WIDE && V != 9 && t.cfg == CFG_F128)
            gemm_tile_fast<V, 128, 128>(p, (int64_t)t.tm * 128, (int64_t)t.tn * 128, 0, d.K, 0, smem);
        else
            gemm_tile_fast<V, 64, 64>(p, (int64_t)t.tm * 64, (int64_t)t.tn * 64, 0, d.K, 0, smem);
    }
}

// WIDE = false: only the 64x64 tile is compiled in (fewer registers, more
// resident workgroups); WIDE = true: all four tile shapes.
template <int V, bool WIDE>
__global__ void __launch_bounds__(256, 1)
persistent_gemm_kernel(const bfx_gemm_desc *__restrict__ probs,
                       const TileItem *__restrict__ tiles, int64_t ntiles, uint32_t *counter) {
    extern __shared__ __align__(16) uint16_t smem[];
    __shared__ int64_t s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t idx = s_idx;
        __syncthreads();
        if (idx >= ntiles) break;
        const TileItem t = tiles[idx];
        const bfx_gemm_desc d = probs[t.prob];
        const GemmParams p = desc_params(d);
        if constexpr (!WIDE) {
            gemm_tile<V, 64, 64, 2, 2>(p, (int64_t)t.tm * 64, (int64_t)t.tn * 64, 0, d.K, 0, smem);
        } else {
            switch (t.cfg) {
                case CFG_64x64:
                    gemm_tile<V, 64, 64, 2, 2>(p, (int64_t)t.tm * 64, (int64_t)t.tn * 64, 0, d.K, 0, smem);
                    break;
                case CFG_128x128:
                    gemm_tile<V, 128, 128, 2, 2>(p, (int64_t)t.tm * 128, (int64_t)t.tn * 128, 0, d.K, 0, smem);
                    break;
                case CFG_128x64:
                    gemm_tile<V, 128, 64, 2, 2>(p, (int64_t)t.tm * 128, (int64_t)t.tn * 64, 0, d.K, 0, smem);
                    break;
                default:
                    gemm_tile<V, 64, 128, 2, 2>(p, (int64_t)t.tm * 64, (int64_t)t.tn * 128, 0, d.K, 0, smem);
                    break;
            }
        }
    }
}

}  // namespace bfx

struct bfx_plan {
    int variant = 6;
    int64_t count = 0, ntiles = 0;
    // [0]: wave-specialised kernel, [1]: general engine kernel
    int64_t n_list[2] = {0, 0};
    bool wide[2] = {false, false};
    size_t lds[2] = {0, 0};
    int grid[2] = {0, 0};
    const void *kern[2] = {nullptr, nullptr};
    std::vector<bfx_gemm_desc> h_probs;
    bfx_gemm_desc *d_probs = nullptr;
    bfx::TileItem *d_tiles = nullptr;   // fast list, then general list
    uint32_t *d_counter = nullptr;      // [0] fast, [1] general
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace bfx {
namespace {

// Tuning table: {"arch": ..., "variant": V, "entries": [{"m": 64, "n": 128,
// "tile": 2}, ...]} where m/n are bucket upper bounds (64, 128, 256, 512) and
// tile indexes cfg_bm/cfg_bn.  Unknown keys are ignored.
bool parse_table(const char *path, int variant, int table[4][4]) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    auto int_after = [&](size_t from, size_t to, const char *key, long &out) {
        const std::string k = std::string("\"") + key + "\"";
        size_t p = s.find(k, from);
        if (p == std::string::npos || p >= to) return false;
        p = s.find(':', p + k.size());
        if (p == std::string::npos || p >= to) return false;
        out = std::strtol(s.c_str() + p + 1, nullptr, 10);
        return true;
    };
    long v = variant;
    const size_t ent = s.find("\"entries\"");
    if (ent == std::string::npos) return false;
    int_after(0, ent, "variant", v);
    if (v != variant) return false;
    size_t pos = ent;
    bool any = false;
    for (;;) {
        const size_t a = s.find('{', pos);
        if (a == std::string::npos) break;
        const size_t b = s.find('}', a);
        if (b == std::string::npos) break;
        long m, n, t;
        if (int_after(a, b, "m", m) && int_after(a, b, "n", n) && int_after(a, b, "tile", t) &&
            t >= 0 && t < NCFG) {
            table[bucket(m)][bucket(n)] = (int)t;
            any = true;
        }
        pos = b + 1;
    }
    return any;
}

// Whether the wave-specialised engine can take the problem (as fast_ok of
// the one-problem path, with the whole K in one range).
bool desc_fast(const bfx_gemm_desc &d) {
    return d.K > 0 && d.K % 4 == 0 && d.N % 4 == 0 && ((uintptr_t)d.A % 16 == 0) && d.lda % 4 == 0 &&
           ((uintptr_t)d.B % 16 == 0) && d.ldb % 4 == 0 && ((uintptr_t)d.C % 4 == 0) &&
           128 * d.lda * 4 < (int64_t(1) << 31) && d.K * d.ldb * 4 < (int64_t(1) << 31);
}

int default_cfg(const bfx_gemm_desc &d) {
    if (desc_fast(d)) return (d.M >= 256 && d.N >= 256) ? CFG_F128 : CFG_F64;
    if (d.M >= 256 && d.N >= 256) return CFG_128x128;
    if (d.M >= 256 && d.N > 64) return CFG_128x64;
    if (d.N >= 256 && d.M > 64) return CFG_64x128;
    return CFG_64x64;
}

template <int V>
void pick(bfx_plan *p) {
    p->kern[0] = p->wide[0] ? (const void *)persistent_fast_kernel<V, true>
                            : (const void *)persistent_fast_kernel<V, false>;
    p->lds[0] = p->wide[0] ? fast_lds_bytes<V, 128, 128>() : fast_lds_bytes<V, 64, 64>();
    p->kern[1] = p->wide[1] ? (const void *)persistent_gemm_kernel<V, true>
                            : (const void *)persistent_gemm_kernel<V, false>;
    p->lds[1] = p->wide[1] ? tile_lds_bytes<V, 128, 128>() : tile_lds_bytes<V, 64, 64>();
}

void plan_free(bfx_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_probs) (void)hipFree(p->d_probs);
    if (p->d_tiles) (void)hipFree(p->d_tiles);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_ws) (void)hipFree(p->d_ws);
    delete p;
}

}  // namespace
}  // namespace bfx

extern "C" int bfx_gemm_batched_plan_create(int variant, int64_t count, const bfx_gemm_desc *descs,
                                            const char *tune_table, bfx_plan **out) {
    using namespace bfx;
    if (variant != 1 && variant != 3 && variant != 6 && variant != 9) return -1;
    if (count < 0) return -2;
    if (count > 0 && !descs) return -3;
    if (!out) return -4;
    *out = nullptr;
    for (int64_t i = 0; i < count; ++i) {
        const bfx_gemm_desc &d = descs[i];
        const bool bad = d.M < 0 || d.N < 0 || d.K < 0 || d.lda < (d.K > 1 ? d.K : 1) ||
                         d.ldb < (d.N > 1 ? d.N : 1) || d.ldc < (d.N > 1 ? d.N : 1) ||
                         (d.M > 0 && d.N > 0 && (!d.C || (d.K > 0 && (!d.A || !d.B))));
        if (bad) {
            char buf[128];
            std::snprintf(buf, sizeof buf, "bfx_gemm_batched_plan_create: descriptor %lld invalid",
                          (long long)i);
            set_error(buf);
            return (int)(-(100 + (i < 1000000 ? i : 1000000)));
        }
    }
    int table[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) table[a][b] = -1;
    if (tune_table && tune_table[0]) parse_table(tune_table, variant, table);

    bfx_plan *p = new bfx_plan();
    p->variant = variant;
    p->count = count;
    p->h_probs.assign(descs, descs + count);
    std::vector<TileItem> tiles[2];
    std::vector<double> cost[2];
    for (int64_t i = 0; i < count; ++i) {
        const bfx_gemm_desc &d = descs[i];
        if (d.M == 0 || d.N == 0) continue;
        int cfg = table[bucket(d.M)][bucket(d.N)];
        if (cfg < 0 || (cfg_fast(cfg) && !desc_fast(d))) cfg = default_cfg(d);
        // x9 with both wave-specialised widths in one kernel exceeds the
        // register file; its batches use the 64-wide tile only
        if (variant == 9 && cfg == CFG_F128) cfg = CFG_F64;
        const int L = cfg_fast(cfg) ? 0 : 1;
        if (cfg != CFG_64x64 && cfg != CFG_F64) p->wide[L] = true;
        const int64_t tm = ceil_div(d.M, cfg_bm[cfg]), tn = ceil_div(d.N, cfg_bn[cfg]);
        const double c = (double)cfg_bm[cfg] * cfg_bn[cfg] * (double)(ceil_div(d.K, BK) + 2);
        for (int64_t a = 0; a < tm; ++a)
            for (int64_t b = 0; b < tn; ++b) {
                tiles[L].push_back(TileItem{(int32_t)i, (int32_t)a, (int32_t)b, cfg});
                cost[L].push_back(c);
            }
        const size_t ws = gemm_ws_bytes(variant, d.M, d.N, d.K);
        if (ws > p->ws_bytes) p->ws_bytes = ws;
    }
    // LPT order within each list; the fast list first in device memory
    std::vector<TileItem> sorted;
    for (int L = 0; L < 2; ++L) {
        std::vector<size_t> order(tiles[L].size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return cost[L][a] > cost[L][b]; });
        for (size_t i = 0; i < order.size(); ++i) sorted.push_back(tiles[L][order[i]]);
        p->n_list[L] = (int64_t)order.size();
    }
    p->ntiles = (int64_t)sorted.size();

    int rc = BFX_OK;
    auto fail = [&](hipError_t e, const char *what) {
        rc = hip_fail(e, what);
        plan_free(p);
        return rc;
    };
    hipError_t e;
    if ((e = hipMalloc(&p->d_probs, sizeof(bfx_gemm_desc) * (count > 0 ? count : 1))) != hipSuccess)
        return fail(e, "hipMalloc(plan descs)");
    if ((e = hipMalloc(&p->d_tiles, sizeof(TileItem) * (sorted.empty() ? 1 : sorted.size()))) != hipSuccess)
        return fail(e, "hipMalloc(plan tiles)");
    if ((e = hipMalloc(&p->d_counter, 256)) != hipSuccess) return fail(e, "hipMalloc(plan counter)");
    if (p->ws_bytes && (e = hipMalloc(&p->d_ws, p->ws_bytes)) != hipSuccess)
        return fail(e, "hipMalloc(plan workspace)");
    if (count > 0 && (e = hipMemcpy(p->d_probs, descs, sizeof(bfx_gemm_desc) * count,
                                    hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy(plan descs)");
    if (!sorted.empty() && (e = hipMemcpy(p->d_tiles, sorted.data(), sizeof(TileItem) * sorted.size(),
                                          hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "hipMemcpy(plan tiles)");

    switch (variant) {
        case 1: pick<1>(p); break;
        case 3: pick<3>(p); break;
        case 6: pick<6>(p); break;
        default: pick<9>(p); break;
    }
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return fail(e, "hipDeviceGetAttribute");
    for (int L = 0; L < 2; ++L) {
        if (p->n_list[L] == 0) continue;
        const int threads = L == 0 ? 512 : 256;
        if ((e = hipFuncSetAttribute(p->kern[L], hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)p->lds[L])) != hipSuccess)
            return fail(e, "hipFuncSetAttribute(persistent)");
        int per_cu = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p->kern[L], threads, p->lds[L])) !=
            hipSuccess)
            return fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        if (per_cu < 1) per_cu = 1;
        p->grid[L] = cus * per_cu;
    }
    if ((e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) != hipSuccess)
        return fail(e, "hipStreamCreate(plan)");
    *out = p;
    return BFX_OK;
}

extern "C" int bfx_plan_launch(bfx_plan *p, void *stream) {
    using namespace bfx;
    if (!p) return -1;
    if (p->ntiles == 0) return BFX_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!p->exec) {
        BFX_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(plan_zero_counter, dim3(1), dim3(64), 0, p->cap, p->d_counter);
        hipError_t el = hipGetLastError();
        for (int L = 0; L < 2 && el == hipSuccess; ++L) {
            if (p->n_list[L] == 0) continue;
            TileItem *list = p->d_tiles + (L == 0 ? 0 : p->n_list[0]);
            uint32_t *cnt = p->d_counter + L;
            void *args[] = {&p->d_probs, &list, &p->n_list[L], &cnt};
            el = hipLaunchKernel(p->kern[L], dim3(p->grid[L]), dim3(L == 0 ? 512 : 256), args,
                                 p->lds[L], p->cap);
        }
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(p->cap, &g);
        if (el != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(el, "persistent kernel capture");
        }
        if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
        p->graph = g;
        BFX_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    BFX_HIP(hipGraphLaunch(p->exec, s));
    return BFX_OK;
}

extern "C" int bfx_plan_launch_per_problem(bfx_plan *p, void *stream) {
    using namespace bfx;
    if (!p) return -1;
    for (const bfx_gemm_desc &d : p->h_probs) {
        const int rc = gemm_launch(p->variant, d.M, d.N, d.K, d.alpha, d.A, d.lda, d.B, d.ldb,
                                   d.beta, d.C, d.ldc, p->d_ws, p->ws_bytes, (hipStream_t)stream);
        if (rc != BFX_OK) return rc;
    }
    return BFX_OK;
}

extern "C" int bfx_plan_info(const bfx_plan *p, int64_t *tiles, int64_t *problems) {
    if (!p) return -1;
    if (tiles) *tiles = p->ntiles;
    if (problems) *problems = p->count;
    return BFX_OK;
}

extern "C" int bfx_plan_destroy(bfx_plan *p) {
    if (!p) return -1;
    bfx::plan_free(p);
    return BFX_OK;
}
