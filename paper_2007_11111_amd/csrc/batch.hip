// batch.hip -- fglt_batch: net frequencies of many small graphs (n <= 512)
// in one launch over a block-diagonal CSR.
//
// One workgroup owns one graph and holds its whole adjacency A as an LDS
// bitmap (n x ceil(n/64) words, at most 32 KiB).  Every Table I quantity then
// reduces to AND + popcount over rows:
//   C3(i,j) = |a_i & a_j| on edges, P2(i,k) = |a_i & a_k| off the diagonal,
//   q_ij = a_i & a_j, and q_ij' A q_ij counts edges inside q_ij.
// The graphs are visited largest first (a device-side counting sort by size),
// so the long graphs start early and the short ones fill the tail.  No
// device memory is allocated and the host never waits, so the launch
// sequence can be captured into a HIP graph and replayed.
#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "raw.h"

namespace fglt {

static constexpr int BMAX = FGLT_BATCH_MAX_N;  // 512
static constexpr int BW = BMAX / 64;           // 8 words per row at most

struct BatchWs {
    i32* order;    // [G] graph ids, largest first
    u32* status;   // [4] status word
    i32* hist;     // [BMAX + 2] size histogram
};

static BatchWs carve_batch(Carver& c, i64 G) {
    BatchWs w{};
    w.status = c.take<u32>(4);
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
    if (threadIdx.x == 0) status[0] = 0;
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

template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_batch_graph(const i64* __restrict__ vtx, const i64* __restrict__ off,
                                                         const i32* __restrict__ idx, const i32* __restrict__ order,
                                                         i64 G, i64 nnz, i64* __restrict__ out,
                                                         u32* __restrict__ status) {
    __shared__ u64 A[BMAX * BW];
    __shared__ i32 sdeg[BMAX];
    __shared__ i32 sp2[BMAX];
    __shared__ i32 sc3[BMAX];
    __shared__ u32 bad;
    const i64 g = order[blockIdx.x];
    const i64 v0 = vtx[g];
    const int n = (int)(vtx[g + 1] - v0);
    if (n <= 0 || n > BMAX) {
        if (threadIdx.x == 0 && n > BMAX) atomicOr(status, ERR_RANGE);
        return;
    }
    const int W = (n + 63) >> 6;
    for (int q = threadIdx.x; q < n * W; q += THREADS) A[q] = 0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    // 1. adjacency bitmap; contract checks (range, self-loop, duplicate)
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const i64 b = off[v0 + i], e = off[v0 + i + 1];
        int len = 0;
        if (b < 0 || e > nnz || e < b || e - b > n) {
            atomicOr(&bad, ERR_RANGE);
        } else {
            for (i64 q = b; q < e; ++q) {
                const i64 j = (i64)idx[q] - v0;
                if (j < 0 || j >= n) {
                    atomicOr(&bad, ERR_RANGE);
                    continue;
                }
                if (j == i) {
                    atomicOr(&bad, ERR_SELFLOOP);
                    continue;
                }
                atomicOr((unsigned long long*)&A[i * W + (j >> 6)], 1ull << (j & 63));
                ++len;
            }
        }
        sdeg[i] = len;
    }
    __syncthreads();
    // 2. degrees (duplicates show as popcount below the row length), symmetry
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const u64* ai = A + i * W;
        int d = 0;
        for (int z = 0; z < W; ++z) d += __popcll(ai[z]);
        if (d != sdeg[i]) atomicOr(&bad, ERR_DUP);
        for (int z = 0; z < W; ++z) {
            u64 word = ai[z];
            while (word) {
                const int j = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                if (!((A[j * W + (i >> 6)] >> (i & 63)) & 1ull)) atomicOr(&bad, ERR_ASYM);
            }
        }
        sdeg[i] = d;
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) atomicOr(status, bad);
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
                sumd += sdeg[j];
                c3x2 += popc_and(ai, A + j * W, W);
            }
        }
        sp2[i] = sumd - sdeg[i];
        sc3[i] = c3x2 >> 1;
    }
    __syncthreads();
    // 4. the rest of Table I, Table II, store
    for (int i = threadIdx.x; i < n; i += THREADS) {
        const u64* ai = A + i * W;
        const i64 d = sdeg[i];
        i64 ap2 = 0, ac3 = 0, s7 = 0, d10 = 0, d14 = 0, d13 = 0, k4 = 0;
        u64 hop[BW];
        for (int z = 0; z < W; ++z) hop[z] = 0;
        for (int z = 0; z < W; ++z) {
            u64 word = ai[z];
            while (word) {
                const int j = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                const u64* aj = A + j * W;
                const i64 dj = sdeg[j];
                ap2 += sp2[j];
                ac3 += sc3[j];
                s7 += (dj - 1) * (dj - 2) / 2;
                const i64 t = popc_and(ai, aj, W);  // C3(i, j)
                d10 += t * (dj - 2);
                d14 += t * (t - 1) / 2;
                for (int y = 0; y < W; ++y) hop[y] |= aj[y];
                // triangles (i, j, k), k > j, k in q_ij
                for (int y = z; y < W; ++y) {
                    u64 q = ai[y] & aj[y];
                    if (y == z) q &= (j & 63) == 63 ? 0ull : (~0ull << ((j & 63) + 1));
                    while (q) {
                        const int k = y * 64 + __ffsll((long long)q) - 1;
                        q &= q - 1;
                        const u64* ak = A + k * W;
                        d13 += popc_and(aj, ak, W) - 1;  // C3(j, k) - 1
                        // 4-cliques {i, j, k, l} with l > k
                        int kk = 0;
                        for (int x = k >> 6; x < W; ++x) {
                            u64 r = ai[x] & aj[x] & ak[x];
                            if (x == (k >> 6)) r &= (k & 63) == 63 ? 0ull : (~0ull << ((k & 63) + 1));
                            kk += __popcll(r);
                        }
                        k4 += kk;
                    }
                }
            }
        }
        // 4-cycles: P2(i, k) = |a_i & a_k| over k two hops away, k != i
        hop[i >> 6] &= ~(1ull << (i & 63));
        i64 c4 = 0;
        for (int z = 0; z < W; ++z) {
            u64 word = hop[z];
            while (word) {
                const int k = z * 64 + __ffsll((long long)word) - 1;
                word &= word - 1;
                const i64 c = popc_and(ai, A + k * W, W);
                c4 += c * (c - 1) / 2;
            }
        }
        const i64 p2 = sp2[i], c3 = sc3[i];
        i64 f[16];
        f[0] = 1;
        f[1] = d;
        f[2] = p2;
        f[3] = d * (d - 1) / 2;
        f[4] = c3;
        f[5] = ap2 - d * (d - 1) - 2 * c3;
        f[6] = d > 0 ? p2 * (d - 1) - 2 * c3 : 0;
        f[7] = s7;
        f[8] = d * (d - 1) * (d - 2) / 6;
        f[9] = ac3 - 2 * c3;
        f[10] = d10;
        f[11] = d >= 2 ? (d - 2) * c3 : 0;
        f[12] = c4;
        f[13] = d13;
        f[14] = d14;
        f[15] = k4;
        raw_to_net16(f);
        i64* o = out + (v0 + i) * 16;
#pragma unroll
        for (int k = 0; k < 16; k += 2) *(longlong2*)(o + k) = make_longlong2(f[k], f[k + 1]);
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

typedef void (*batch_kernel_t)(const i64*, const i64*, const i32*, const i32*, i64, i64, i64*, u32*);

static batch_kernel_t pick_kernel(int threads) {
    switch (threads) {
        case 64: return k_batch_graph<64>;
        case 128: return k_batch_graph<128>;
        case 512: return k_batch_graph<512>;
        case 1024: return k_batch_graph<1024>;
        default: return k_batch_graph<256>;
    }
}

static hipError_t enqueue_batch(hipStream_t s, int threads, i64 G, const i64* vtx, const i64* off, const i32* idx,
                                i64 nnz, i64* net, BatchWs& w) {
    hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, vtx, G, w.order, w.hist, w.status);
    hipLaunchKernelGGL(pick_kernel(threads), dim3((unsigned)G), dim3(threads), 0, s, vtx, off, idx,
                       (const i32*)w.order, G, nnz, net, w.status);
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
    int threads = plan && plan->threads ? plan->threads : 256;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024) return FGLT_EINVAL;
    const bool use_graph = plan && plan->use_graph;
    hipStream_t s = (hipStream_t)stream;
    if (use_graph && s == nullptr) return FGLT_EINVAL;  // the legacy default stream cannot be captured
    Carver c(ws, ws_bytes);
    BatchWs w = carve_batch(c, num_graphs);
    if (!c.ok()) return FGLT_EWORKSPACE;
    if (!use_graph) {
        FGLT_HIP_TRY(enqueue_batch(s, threads, num_graphs, vtx_offsets, offsets, indices, nnz_total, net, w));
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
        hipError_t e = enqueue_batch(s, threads, num_graphs, vtx_offsets, offsets, indices, nnz_total, net, w);
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
        i64* a5 = net;
        u32* a6 = w.status;
        void* args[] = {(void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3, (void*)&G, (void*)&nz, (void*)&a5, (void*)&a6};
        hipKernelNodeParams p{};
        p.func = (void*)pick_kernel(threads);
        p.gridDim = dim3((unsigned)num_graphs);
        p.blockDim = dim3(threads);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        FGLT_HIP_TRY(hipGraphExecKernelNodeSetParams(cg.exec, cg.main_node, &p));
    }
    FGLT_HIP_TRY(hipGraphLaunch(cg.exec, s));
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
            if (it->second.exec) hipGraphExecDestroy(it->second.exec);
            if (it->second.graph) hipGraphDestroy(it->second.graph);
            it = g_cache.erase(it);
        } else {
            ++it;
        }
    }
    return FGLT_OK;
}
