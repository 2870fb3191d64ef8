// batch.hip -- fglt_batch: net frequencies of many small graphs (n <= 512)
// in one launch over a block-diagonal CSR.
//
// One workgroup owns one graph and holds its whole adjacency A as an LDS
// bitmap (n x ceil(n/64) words, at most 32 KiB).  Every Table I quantity then
// reduces to AND + popcount over rows:
//   C3(i,j) = |a_i & a_j| on edges, P2(i,k) = |a_i & a_k| off the diagonal,
//   q_ij = a_i & a_j, and q_ij' A q_ij counts edges inside q_ij.
// The graphs are visited largest first (a device-side counting sort by size)
// through a work queue: a persistent grid of workgroups takes the next graph
// from a device counter, so the long graphs start early and the short ones
// fill the tail.  In the last pass a vertex of degree >= hub_degree is taken
// by a whole wavefront (its lanes split the neighbours and the 2-hop
// candidates), the others by one thread each, so that hubs of preferential-
// attachment graphs do not hold up their workgroup.  No device memory is
// allocated and the host never waits, so the launch sequence can be captured
// into a HIP graph and replayed.  fglt_batch_tune times candidate plans
// (threads, hub degree, workgroups per CU) on the caller's batch.
#include <algorithm>
#include <array>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "raw.h"

namespace fglt {

static constexpr int BMAX = FGLT_BATCH_MAX_N;  // 512
static constexpr int BW = BMAX / 64;           // 8 words per row at most

struct BatchWs {
    i32* order;    // [G] graph ids, largest first
    u32* status;   // [4] status word, then the work queue's head
    i32* hist;     // [BMAX + 2] size histogram
};

static BatchWs carve_batch(Carver& c, i64 G) {
    BatchWs w{};
    w.status = c.take<u32>(4);  // the status word must stay the first piece (fglt_batch_status)
    w.hist = c.take<i32>(BMAX + 2);
    w.order = c.take<i32>(std::max<i64>(G, 1));
    return w;
}

// One workgroup: counting sort of the graphs by decreasing vertex count;
// also clears the status word (kept a kernel so the sequence is capturable).
__global__ void __launch_bounds__(1024) k_batch_order(const i64* __restrict__ vtx, i64 G, i32* __restrict__ order,
                                                      i32* __restrict__ hist, u32* __restrict__ status) {
    __shared__ i32 h[BMAX + 2];
    for (int t = threadIdx.x; t < BMAX + 2; t += blockDim.x) h[t] = 0;
    if (threadIdx.x == 0) {
        status[0] = 0;
        status[1] = 0;  // the work queue's head
    }
    __syncthreads();
    for (i64 g = threadIdx.x; g < G; g += blockDim.x) {
        i64 n = vtx[g + 1] - vtx[g];
        n = n < 0 ? 0 : (n > BMAX ? BMAX + 1 : n);
        atomicAdd(&h[BMAX + 1 - n], 1);  // bucket 0 = largest
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        i32 run = 0;
        for (int b = 0; b < BMAX + 2; ++b) {
            const i32 c = h[b];
            h[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (i64 g = threadIdx.x; g < G; g += blockDim.x) {
        i64 n = vtx[g + 1] - vtx[g];
        n = n < 0 ? 0 : (n > BMAX ? BMAX + 1 : n);
        const i32 pos = atomicAdd(&h[BMAX + 1 - n], 1);
        order[pos] = (i32)g;
    }
    (void)hist;
}

__device__ __forceinline__ int popc_and(const u64* a, const u64* b, int W) {
    int s = 0;
    for (int z = 0; z < W; ++z) s += __popcll(a[z] & b[z]);
    return s;
}

// Sums of the last pass of vertex i over those of its neighbours j whose
// index among them is congruent to `part` modulo `nparts` (a power of two):
// A p2, A c3, A C(p1-1, 2), C3 (p1-2), C(C3, 2), the diamonds off-cord
// sum_{k in q_ij, k > j} (C3(j, k) - 1) and the 4-cliques {i, j, k, l} with
// l > k > j; `hop` collects their rows (the 2-hop candidates).
struct VSums {
    i64 ap2, ac3, s7, d10, d14, d13, k4;
};

__device__ __forceinline__ void nbr_sums(const u64* A, int W, int i, const i32* sdeg, const i32* sp2, const i32* sc3,
                                         int part, int nparts, VSums& v, u64* hop) {
    const u64* ai = A + i * W;
    int t = 0;
    for (int z = 0; z < W; ++z) {
        u64 word = ai[z];
        while (word) {
            const int j = z * 64 + __ffsll((long long)word) - 1;
            word &= word - 1;
            if ((t++ & (nparts - 1)) != part) continue;
            const u64* aj = A + j * W;
            const i64 dj = sdeg[j];
            v.ap2 += sp2[j];
            v.ac3 += sc3[j];
            v.s7 += (dj - 1) * (dj - 2) / 2;
            const i64 c = popc_and(ai, aj, W);  // C3(i, j)
            v.d10 += c * (dj - 2);
            v.d14 += c * (c - 1) / 2;
            for (int y = 0; y < W; ++y) hop[y] |= aj[y];
            // triangles (i, j, k), k > j, k in q_ij
            for (int y = z; y < W; ++y) {
                u64 q = ai[y] & aj[y];
                if (y == z) q &= (j & 63) == 63 ? 0ull : (~0ull << ((j & 63) + 1));
                while (q) {
                    const int k = y * 64 + __ffsll((long long)q) - 1;
                    q &= q - 1;
                    const u64* ak = A + k * W;
                    v.d13 += popc_and(aj, ak, W) - 1;  // C3(j, k) - 1
                    // 4-cliques {i, j, k, l} with l > k
                    int kk = 0;
                    for (int x = k >> 6; x < W; ++x) {
                        u64 r = ai[x] & aj[x] & ak[x];
                        if (x == (k >> 6)) r &= (k & 63) == 63 ? 0ull : (~0ull << ((k & 63) + 1));
                        kk += __popcll(r);
                    }
                    v.k4 += kk;
                }
            }
        }
    }
}

// 4-cycles at i: sum of C(P2(i, k), 2) over the 2-hop candidates k != i
// (P2(i, k) = |a_i & a_k|); with nparts == 64, lane `part` takes the
// candidates k = 64 z + part.
__device__ __forceinline__ i64 c4_sum(const u64* A, int W, int i, const u64* hop, int part, int nparts) {
    const u64* ai = A + i * W;
    i64 c4 = 0;
    if (nparts == 1) {
        for (int z = 0; z < W; ++z) {
            u64 word = hop[z];
            while (word) {
                const int k = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                const i64 c = popc_and(ai, A + k * W, W);
                c4 += c * (c - 1) / 2;
            }
        }
    } else {
        for (int z = 0; z < W; ++z) {
            if (!((hop[z] >> part) & 1ull)) continue;
            const i64 c = popc_and(ai, A + (z * 64 + part) * W, W);
            c4 += c * (c - 1) / 2;
        }
    }
    return c4;
}

// Table I then Table II for one vertex, stored as a 128-byte row.
__device__ __forceinline__ void batch_store(i64* __restrict__ o, i64 d, i64 p2, i64 c3, const VSums& v, i64 c4) {
    i64 f[16];
    f[0] = 1;
    f[1] = d;
    f[2] = p2;
    f[3] = d * (d - 1) / 2;
    f[4] = c3;
    f[5] = v.ap2 - d * (d - 1) - 2 * c3;
    f[6] = d > 0 ? p2 * (d - 1) - 2 * c3 : 0;
    f[7] = v.s7;
    f[8] = d * (d - 1) * (d - 2) / 6;
    f[9] = v.ac3 - 2 * c3;
    f[10] = v.d10;
    f[11] = d >= 2 ? (d - 2) * c3 : 0;
    f[12] = c4;
    f[13] = v.d13;
    f[14] = v.d14;
    f[15] = v.k4;
    raw_to_net16(f);
#pragma unroll
    for (int k = 0; k < 16; k += 2) *(longlong2*)(o + k) = make_longlong2(f[k], f[k + 1]);
}

__device__ __forceinline__ u64 wave_or64(u64 x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x |= (u64)__shfl_xor((long long)x, off, WAVE);
    return x;
}

struct BatchLds {
    u64 A[BMAX * BW];
    i32 sdeg[BMAX];
    i32 sp2[BMAX];
    i32 sc3[BMAX];
    u32 bad;
    i32 sg;
};

// One graph by one workgroup.  Returns early (uniformly over the block) for
// an empty or oversized graph or one that breaks the contract.
template <int THREADS>
__device__ __forceinline__ void batch_one(BatchLds& S, i64 g, const i64* __restrict__ vtx,
                                          const i64* __restrict__ off, const i32* __restrict__ idx, i64 nnz,
                                          int hub_deg, i64* __restrict__ out, u32* __restrict__ status) {
    u64* const A = S.A;
    const i64 v0 = vtx[g];
    const int n = (int)(vtx[g + 1] - v0);
    if (n <= 0 || n > BMAX) {
        if (threadIdx.x == 0 && n > BMAX) atomicOr(status, ERR_RANGE);
        return;
    }
    const int W = (n + 63) >> 6;
    for (int q = threadIdx.x; q < n * W; q += THREADS) A[q] = 0;
    if (threadIdx.x == 0) S.bad = 0;
    __syncthreads();
    // 1. adjacency bitmap; contract checks (range, self-loop, duplicate)
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const i64 b = off[v0 + i], e = off[v0 + i + 1];
        int len = 0;
        if (b < 0 || e > nnz || e < b || e - b > n) {
            atomicOr(&S.bad, ERR_RANGE);
        } else {
            for (i64 q = b; q < e; ++q) {
                const i64 j = (i64)idx[q] - v0;
                if (j < 0 || j >= n) {
                    atomicOr(&S.bad, ERR_RANGE);
                    continue;
                }
                if (j == i) {
                    atomicOr(&S.bad, ERR_SELFLOOP);
                    continue;
                }
                atomicOr((unsigned long long*)&A[i * W + (j >> 6)], 1ull << (j & 63));
                ++len;
            }
        }
        S.sdeg[i] = len;
    }
    __syncthreads();
    // 2. degrees (duplicates show as popcount below the row length), symmetry
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const u64* ai = A + i * W;
        int d = 0;
        for (int z = 0; z < W; ++z) d += __popcll(ai[z]);
        if (d != S.sdeg[i]) atomicOr(&S.bad, ERR_DUP);
        for (int z = 0; z < W; ++z) {
            u64 word = ai[z];
            while (word) {
                const int j = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                if (!((A[j * W + (i >> 6)] >> (i & 63)) & 1ull)) atomicOr(&S.bad, ERR_ASYM);
            }
        }
        S.sdeg[i] = d;
    }
    __syncthreads();
    if (S.bad) {
        if (threadIdx.x == 0) atomicOr(status, S.bad);
        return;  // the whole block leaves together
    }
    // 3. per-vertex first pass: p2, c3 (needed by neighbours in pass 4)
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const u64* ai = A + i * W;
        int sumd = 0, c3x2 = 0;
        for (int z = 0; z < W; ++z) {
            u64 word = ai[z];
            while (word) {
                const int j = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                sumd += S.sdeg[j];
                c3x2 += popc_and(ai, A + j * W, W);
            }
        }
        S.sp2[i] = sumd - S.sdeg[i];
        S.sc3[i] = c3x2 >> 1;
    }
    __syncthreads();
    // 4. the rest of Table I, Table II, store: light vertices one thread each,
    // vertices of degree >= hub_deg one wavefront each
    for (int i = threadIdx.x; i < n; i += THREADS) {
        if (S.sdeg[i] >= hub_deg) continue;
        VSums v{};
        u64 hop[BW];
        for (int z = 0; z < W; ++z) hop[z] = 0;
        nbr_sums(A, W, i, S.sdeg, S.sp2, S.sc3, 0, 1, v, hop);
        hop[i >> 6] &= ~(1ull << (i & 63));
        const i64 c4 = c4_sum(A, W, i, hop, 0, 1);
        batch_store(out + (v0 + i) * 16, S.sdeg[i], S.sp2[i], S.sc3[i], v, c4);
    }
    const int lane = lane_id();
    for (int i = threadIdx.x / WAVE; i < n; i += THREADS / WAVE) {
        if (S.sdeg[i] < hub_deg) continue;  // uniform over the wavefront
        VSums v{};
        u64 hop[BW];
        for (int z = 0; z < W; ++z) hop[z] = 0;
        nbr_sums(A, W, i, S.sdeg, S.sp2, S.sc3, lane, WAVE, v, hop);
        for (int z = 0; z < W; ++z) hop[z] = wave_or64(hop[z]);
        hop[i >> 6] &= ~(1ull << (i & 63));
        i64 c4 = c4_sum(A, W, i, hop, lane, WAVE);
        v.ap2 = wave_sum(v.ap2);
        v.ac3 = wave_sum(v.ac3);
        v.s7 = wave_sum(v.s7);
        v.d10 = wave_sum(v.d10);
        v.d14 = wave_sum(v.d14);
        v.d13 = wave_sum(v.d13);
        v.k4 = wave_sum(v.k4);
        c4 = wave_sum(c4);
        if (lane == 0) batch_store(out + (v0 + i) * 16, S.sdeg[i], S.sp2[i], S.sc3[i], v, c4);
    }
}

// Persistent workgroups: each takes the next graph (largest first) from the
// work queue (status[1], cleared by k_batch_order) until none is left.
template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_batch_graph(const i64* __restrict__ vtx, const i64* __restrict__ off,
                                                         const i32* __restrict__ idx, const i32* __restrict__ order,
                                                         i64 G, i64 nnz, int hub_deg, i64* __restrict__ out,
                                                         u32* __restrict__ status) {
    __shared__ BatchLds S;
    while (true) {
        if (threadIdx.x == 0) S.sg = (i32)atomicAdd(&status[1], 1u);
        __syncthreads();
        const i64 gi = S.sg;
        if (gi >= G) break;  // uniform over the block
        batch_one<THREADS>(S, order[gi], vtx, off, idx, nnz, hub_deg, out, status);
        __syncthreads();  // LDS is reused by the next graph
    }
}

// ---------------------------------------------------------------- HIP graph cache

struct GraphKey {
    hipStream_t stream;
    i64 G;
    int threads;
    bool operator==(const GraphKey& o) const { return stream == o.stream && G == o.G && threads == o.threads; }
};
struct GraphKeyHash {
    size_t operator()(const GraphKey& k) const {
        return std::hash<void*>()((void*)k.stream) ^ (std::hash<i64>()(k.G) * 31) ^ (size_t)k.threads;
    }
};
struct CachedGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t order_node = nullptr, main_node = nullptr;
};
static std::mutex g_cache_mu;
static std::unordered_map<GraphKey, CachedGraph, GraphKeyHash> g_cache;

typedef void (*batch_kernel_t)(const i64*, const i64*, const i32*, const i32*, i64, i64, int, i64*, u32*);

static batch_kernel_t pick_kernel(int threads) {
    switch (threads) {
        case 64: return k_batch_graph<64>;
        case 128: return k_batch_graph<128>;
        case 512: return k_batch_graph<512>;
        case 1024: return k_batch_graph<1024>;
        default: return k_batch_graph<256>;
    }
}

// The resolved execution plan of one call.
struct BatchCfg {
    int threads;
    int hub_deg;      // degree from which a vertex is taken by a wavefront
    unsigned grid;    // persistent workgroups
};

static constexpr int BATCH_CUS = 256;

static BatchCfg batch_cfg(const fglt_batch_plan* plan, i64 G) {
    BatchCfg c{256, BMAX + 1, 0};  // default: one thread per vertex, a workgroup per graph
    int bpc = 64;
    if (plan) {
        if (plan->threads) c.threads = plan->threads;
        if (plan->hub_degree > 0) c.hub_deg = plan->hub_degree;
        if (plan->hub_degree < 0) c.hub_deg = BMAX + 1;  // no wavefront hubs
        if (plan->blocks_per_cu > 0) bpc = plan->blocks_per_cu;
    }
    c.grid = (unsigned)std::max<i64>(1, std::min<i64>(G, (i64)bpc * BATCH_CUS));
    return c;
}

static hipError_t enqueue_batch(hipStream_t s, const BatchCfg& c, i64 G, const i64* vtx, const i64* off,
                                const i32* idx, i64 nnz, i64* net, BatchWs& w) {
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, vtx, G, w.order, w.hist, w.status);
    hipLaunchKernelGGL(pick_kernel(c.threads), dim3(c.grid), dim3(c.threads), 0, s, vtx, off, idx,
                       (const i32*)w.order, G, nnz, c.hub_deg, net, w.status);
    return hipGetLastError();
}

}  // namespace fglt

using namespace fglt;

extern "C" size_t fglt_batch_workspace(int32_t num_graphs, int64_t n_total, int64_t nnz_total) {
    (void)n_total;
    (void)nnz_total;
    if (num_graphs < 0) return 0;
    Carver c(nullptr, 0);
    carve_batch(c, num_graphs);
    return c.used;
}

extern "C" int fglt_batch(int32_t num_graphs, const int64_t* vtx_offsets, const int64_t* vtx_offsets_host,
                          int64_t n_total, int64_t nnz_total, const int64_t* offsets, const int32_t* indices,
                          int64_t* net, const fglt_batch_plan* plan, void* ws, size_t ws_bytes, void* stream) {
    if (num_graphs < 0 || n_total < 0 || nnz_total < 0 || n_total >= ((int64_t)1 << 31)) return FGLT_EINVAL;
    if (num_graphs == 0) return n_total == 0 ? FGLT_OK : FGLT_EINVAL;
    if (!vtx_offsets || !vtx_offsets_host || !offsets || !net || !ws) return FGLT_EINVAL;
    if (nnz_total > 0 && !indices) return FGLT_EINVAL;
    if (vtx_offsets_host[0] != 0 || vtx_offsets_host[num_graphs] != n_total) return FGLT_EINVAL;
    for (int32_t g = 0; g < num_graphs; ++g) {
        const int64_t ng = vtx_offsets_host[g + 1] - vtx_offsets_host[g];
        if (ng < 0) return FGLT_EINVAL;
        if (ng > FGLT_BATCH_MAX_N) return FGLT_EUNSUPPORTED;
    }
    const BatchCfg cfg = batch_cfg(plan, num_graphs);
    const int threads = cfg.threads;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024) return FGLT_EINVAL;
    if (plan && (plan->blocks_per_cu < 0 || plan->blocks_per_cu > 64)) return FGLT_EINVAL;
    const bool use_graph = plan && plan->use_graph;
    hipStream_t s = (hipStream_t)stream;
    if (use_graph && s == nullptr) return FGLT_EINVAL;  // the legacy default stream cannot be captured
    Carver c(ws, ws_bytes);
    BatchWs w = carve_batch(c, num_graphs);
    if (!c.ok()) return FGLT_EWORKSPACE;
    if (!use_graph) {
        FGLT_HIP_TRY(enqueue_batch(s, cfg, num_graphs, vtx_offsets, offsets, indices, nnz_total, net, w));
        return FGLT_OK;
    }
    // Replay a captured graph for (stream, G, threads), with the kernel
    // arguments of this call written into its two kernel nodes.
    std::lock_guard<std::mutex> lock(g_cache_mu);
    GraphKey key{s, num_graphs, threads};
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
        CachedGraph cg;
        FGLT_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_batch(s, cfg, num_graphs, vtx_offsets, offsets, indices, nnz_total, net, w);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) return FGLT_EHIP;
        size_t nn = 0;
        FGLT_HIP_TRY(hipGraphGetNodes(graph, nullptr, &nn));
        std::vector<hipGraphNode_t> nodes(nn);
        FGLT_HIP_TRY(hipGraphGetNodes(graph, nodes.data(), &nn));
        for (auto nd : nodes) {
            hipGraphNodeType ty;
            FGLT_HIP_TRY(hipGraphNodeGetType(nd, &ty));
            if (ty != hipGraphNodeTypeKernel) continue;
            hipKernelNodeParams p;
            FGLT_HIP_TRY(hipGraphKernelNodeGetParams(nd, &p));
            if (p.func == (void*)k_batch_order) cg.order_node = nd;
            else cg.main_node = nd;
        }
        if (!cg.order_node || !cg.main_node) return FGLT_EHIP;
        FGLT_HIP_TRY(hipGraphInstantiate(&cg.exec, graph, nullptr, nullptr, 0));
        cg.graph = graph;
        it = g_cache.emplace(key, cg).first;
    }
    CachedGraph& cg = it->second;
    {
        i64 G = num_graphs;
        const i64* a0 = vtx_offsets;
        i32* a1 = w.order;
        i32* a2 = w.hist;
        u32* a3 = w.status;
        void* args[] = {(void*)&a0, (void*)&G, (void*)&a1, (void*)&a2, (void*)&a3};
        hipKernelNodeParams p{};
        p.func = (void*)k_batch_order;
        p.gridDim = dim3(1);
        p.blockDim = dim3(1024);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        FGLT_HIP_TRY(hipGraphExecKernelNodeSetParams(cg.exec, cg.order_node, &p));
    }
    {
        const i64* a0 = vtx_offsets;
        const i64* a1 = offsets;
        const i32* a2 = indices;
        const i32* a3 = w.order;
        i64 G = num_graphs;
        i64 nz = nnz_total;
        int hd = cfg.hub_deg;
        i64* a5 = net;
        u32* a6 = w.status;
        void* args[] = {(void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3, (void*)&G, (void*)&nz, (void*)&hd,
                        (void*)&a5, (void*)&a6};
        hipKernelNodeParams p{};
        p.func = (void*)pick_kernel(threads);
        p.gridDim = dim3(cfg.grid);
        p.blockDim = dim3(threads);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        FGLT_HIP_TRY(hipGraphExecKernelNodeSetParams(cg.exec, cg.main_node, &p));
    }
    FGLT_HIP_TRY(hipGraphLaunch(cg.exec, s));
    return FGLT_OK;
}

// ---------------------------------------------------------------- autotuner

// Cache key of a tuned plan: the batch's shape and its histogram of graph
// sizes in 16 bins of 32 vertices.
struct TuneKey {
    i64 G, n_total, nnz_total;
    std::array<i64, 16> hist;
    bool operator==(const TuneKey& o) const {
        return G == o.G && n_total == o.n_total && nnz_total == o.nnz_total && hist == o.hist;
    }
};
struct TuneKeyHash {
    size_t operator()(const TuneKey& k) const {
        size_t h = std::hash<i64>()(k.G) ^ (std::hash<i64>()(k.n_total) * 31) ^ (std::hash<i64>()(k.nnz_total) * 131);
        for (i64 x : k.hist) h = h * 1000003u ^ std::hash<i64>()(x);
        return h;
    }
};
static std::mutex g_tune_mu;
static std::unordered_map<TuneKey, fglt_batch_plan, TuneKeyHash> g_tuned;

extern "C" int fglt_batch_tune(int32_t num_graphs, const int64_t* vtx_offsets, const int64_t* vtx_offsets_host,
                               int64_t n_total, int64_t nnz_total, const int64_t* offsets, const int32_t* indices,
                               int64_t* net, void* ws, size_t ws_bytes, int32_t reps, fglt_batch_plan* plan_out,
                               void* stream) {
    if (!plan_out || !vtx_offsets_host || reps < 1 || reps > 100) return FGLT_EINVAL;
    if (num_graphs < 0) return FGLT_EINVAL;
    TuneKey key{num_graphs, n_total, nnz_total, {}};
    for (int32_t g = 0; g < num_graphs; ++g) {
        const int64_t ng = vtx_offsets_host[g + 1] - vtx_offsets_host[g];
        key.hist[(size_t)std::min<int64_t>(15, std::max<int64_t>(0, (ng - 1) / 32))]++;
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *plan_out = it->second;
            return FGLT_OK;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EvGuard {
        hipEvent_t& a;
        hipEvent_t& b;
        ~EvGuard() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    FGLT_HIP_TRY(hipEventCreate(&e0));
    FGLT_HIP_TRY(hipEventCreate(&e1));
    static const int kThreads[] = {128, 256, 512};
    static const int kHub[] = {16, 32, 64, -1};
    static const int kBpc[] = {2, 4, 8, 64};
    fglt_batch_plan best{256, 0, 0, 0};
    float best_ms = -1.f;
    for (int th : kThreads)
        for (int hub : kHub)
            for (int bpc : kBpc) {
                fglt_batch_plan p{th, hub, bpc, 0};
                int st = fglt_batch(num_graphs, vtx_offsets, vtx_offsets_host, n_total, nnz_total, offsets, indices,
                                    net, &p, ws, ws_bytes, stream);  // warm-up (and argument checks)
                if (st) return st;
                std::vector<float> t;
                for (int r = 0; r < reps; ++r) {
                    FGLT_HIP_TRY(hipEventRecord(e0, s));
                    st = fglt_batch(num_graphs, vtx_offsets, vtx_offsets_host, n_total, nnz_total, offsets, indices,
                                    net, &p, ws, ws_bytes, stream);
                    if (st) return st;
                    FGLT_HIP_TRY(hipEventRecord(e1, s));
                    FGLT_HIP_TRY(hipEventSynchronize(e1));
                    float ms = 0.f;
                    FGLT_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                    t.push_back(ms);
                }
                std::sort(t.begin(), t.end());
                const float med = t[t.size() / 2];
                if (best_ms < 0.f || med < best_ms) {
                    best_ms = med;
                    best = p;
                }
            }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = best;
    }
    *plan_out = best;
    return FGLT_OK;
}

extern "C" int fglt_batch_status(const void* ws, void* stream) {
    if (!ws) return FGLT_EINVAL;
    u32 st = 0;
    // the status word is the first piece of the batch workspace
    FGLT_HIP_TRY(hipMemcpyAsync(&st, ws, sizeof(u32), hipMemcpyDeviceToHost, (hipStream_t)stream));
    FGLT_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return st ? FGLT_ENOTCANON : FGLT_OK;
}

extern "C" int fglt_batch_release(void* stream) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (stream == nullptr || it->first.stream == (hipStream_t)stream) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
            it = g_cache.erase(it);
        } else {
            ++it;
        }
    }
    return FGLT_OK;
}
