// totals.hip -- graph-level totals of the net frequencies: for each graph of
// a batch and each orbit k, the number of induced copies of orbit k's
// graphlet.  The net frequency f_k(v) counts the induced copies of that
// graphlet in which v lies in orbit k (the problem description of the
// graphlet transform and the Sigma_16 section; the orbits of Fig. 1), so the sum
// of column k over a graph counts every copy once per vertex of the copy in
// orbit k: m_k times.
#include <algorithm>

#include "raw.h"

namespace fglt {

// m_k: vertices of orbit k's graphlet that lie in orbit k -- node, edge,
// path P3 (ends, centre), triangle, path P4 (ends, inner), claw (leaves,
// centre), paw (tail, the two plain triangle vertices, the joint), 4-cycle,
// diamond (the two kinds of vertex), 4-clique.
__device__ __forceinline__ i64 orbit_nodes(int k) {
    constexpr unsigned long long packed = 0x4224121132231221ull;  // nibble k = m_k
    return (i64)((packed >> (4 * k)) & 0xfull);
}

static constexpr int NORB = 16;  // orbits of Sigma_16
static constexpr int TOT_THREADS = 256;

// Workgroup (g, p) sums the rows of part p (of gridDim.y) of graph g.  One
// part: the totals are written divided by m_k; several: the sums are added
// to zeroed totals, and k_totals_div divides them afterwards.
__global__ void __launch_bounds__(TOT_THREADS) k_totals_sum(const i64* __restrict__ off, i64 n_total,
                                                            const i64* __restrict__ net, i64* __restrict__ totals) {
    __shared__ i64 part[TOT_THREADS / WAVE][NORB];
    const i64 g = blockIdx.x;
    const i64 lo = std::min(std::max(off[g], (i64)0), n_total);
    const i64 hi = std::min(std::max(off[g + 1], lo), n_total);
    const i64 len = hi - lo, P = gridDim.y;
    const i64 b0 = lo + len * blockIdx.y / P, b1 = lo + len * (blockIdx.y + 1) / P;
    i64 acc[NORB];
#pragma unroll
    for (int k = 0; k < NORB; ++k) acc[k] = 0;
    for (i64 v = b0 + threadIdx.x; v < b1; v += TOT_THREADS) {
#pragma unroll
        for (int k = 0; k < NORB; ++k) acc[k] += net[v * NORB + k];
    }
    const int wv = threadIdx.x / WAVE, l = lane_id();
#pragma unroll
    for (int k = 0; k < NORB; ++k) {
        const i64 s = wave_sum(acc[k]);
        if (l == 0) part[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NORB) {
        const int k = threadIdx.x;
        i64 s = 0;
        for (int w = 0; w < TOT_THREADS / WAVE; ++w) s += part[w][k];
        if (P == 1) totals[g * NORB + k] = s / orbit_nodes(k);
        else if (s) atomicAdd((unsigned long long*)&totals[g * NORB + k], (unsigned long long)s);
    }
}

__global__ void k_totals_fill0(i64* __restrict__ p, i64 cnt) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (i64)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_totals_div(i64* __restrict__ totals, i64 cnt) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (i64)gridDim.x * blockDim.x)
        totals[i] /= orbit_nodes((int)(i % NORB));
}

}  // namespace fglt

using namespace fglt;

extern "C" int fglt_totals(int64_t num_graphs, const int64_t* vtx_offsets, int64_t n_total, const int64_t* net,
                           int64_t* totals, void* stream) {
    if (num_graphs < 0 || n_total < 0 || num_graphs >= ((int64_t)1 << 31)) return FGLT_EINVAL;
    if (num_graphs == 0) return FGLT_OK;
    if (!vtx_offsets || !totals || (n_total > 0 && !net)) return FGLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const i64 G = num_graphs;
    // parts per graph: about 8192 rows each, at most 1024 (a single large graph
    // spreads over the GPU; a batch of small graphs takes one workgroup each)
    const i64 parts = std::min<i64>(1024, std::max<i64>(1, ceil_div(n_total, G * 8192)));
    const i64 cells = G * NORB;
    if (parts > 1)
        hipLaunchKernelGGL(k_totals_fill0, dim3(grid_for(cells, TOT_THREADS, 4096)), dim3(TOT_THREADS), 0, s, totals, cells);
    hipLaunchKernelGGL(k_totals_sum, dim3((unsigned)G, (unsigned)parts), dim3(TOT_THREADS), 0, s, vtx_offsets,
                       n_total, net, totals);
    if (parts > 1)
        hipLaunchKernelGGL(k_totals_div, dim3(grid_for(cells, TOT_THREADS, 4096)), dim3(TOT_THREADS), 0, s, totals, cells);
    FGLT_HIP_TRY(hipGetLastError());
    return FGLT_OK;
}
