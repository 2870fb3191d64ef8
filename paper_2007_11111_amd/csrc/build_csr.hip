// build_csr.hip -- canonical adjacency of a simple undirected graph from an
// edge list: both directions, self-loops dropped, duplicates dropped, rows
// sorted (the graph model of Section I of the paper: symmetric 0/1 A).
//
// Pipeline: per-vertex counts (atomics) -> exclusive scan -> scatter with
// per-row cursors -> segmented sort of each row -> keep-flags for the first
// of each run of equal entries -> scan of the flags -> compaction.
#include <algorithm>

#include "common.h"

namespace fglt {

__global__ void k_bc_count(const i32* __restrict__ src, const i32* __restrict__ dst, i64 E, i64 n,
                           i32* __restrict__ cnt, u32* __restrict__ err) {
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < E; t += (i64)gridDim.x * blockDim.x) {
        const i32 a = src[t], b = dst[t];
        if (a < 0 || b < 0 || (i64)a >= n || (i64)b >= n) {
            atomicOr(err, ERR_RANGE);
            continue;
        }
        if (a == b) continue;
        atomicAdd(&cnt[a], 1);
        atomicAdd(&cnt[b], 1);
    }
}

__global__ void k_bc_scatter(const i32* __restrict__ src, const i32* __restrict__ dst, i64 E, i64 n,
                             const i64* __restrict__ toff, i32* __restrict__ cursor, i32* __restrict__ tidx) {
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < E; t += (i64)gridDim.x * blockDim.x) {
        const i32 a = src[t], b = dst[t];
        if (a < 0 || b < 0 || (i64)a >= n || (i64)b >= n || a == b) continue;
        const i32 pa = atomicAdd(&cursor[a], 1);
        tidx[toff[a] + pa] = b;
        const i32 pb = atomicAdd(&cursor[b], 1);
        tidx[toff[b] + pb] = a;
    }
}

// keep[p] = 1 for the first entry of every run of equal values inside a row.
__global__ void k_bc_keep(const i32* __restrict__ tidx, const i64* __restrict__ toff, i64 n,
                          i32* __restrict__ keep) {
    const i64 total = toff[n];
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (i64)gridDim.x * blockDim.x)
        keep[p] = (p == 0 || tidx[p] != tidx[p - 1]) ? 1 : 0;
}

__global__ void k_bc_rowstart(const i64* __restrict__ toff, i64 n, i32* __restrict__ keep) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        const i64 b = toff[r];
        if (toff[r + 1] > b) keep[b] = 1;
    }
}

__global__ void k_bc_zero_tail(i32* __restrict__ keep, const i64* __restrict__ toff, i64 n, i64 cap) {
    for (i64 p = toff[n] + (i64)blockIdx.x * blockDim.x + threadIdx.x; p < cap; p += (i64)gridDim.x * blockDim.x)
        keep[p] = 0;
}

__global__ void k_bc_compact(const i32* __restrict__ tidx, const i32* __restrict__ keep,
                             const i64* __restrict__ pos, const i64* __restrict__ toff, i64 n,
                             i32* __restrict__ indices) {
    const i64 total = toff[n];
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < total; p += (i64)gridDim.x * blockDim.x)
        if (keep[p]) indices[pos[p]] = tidx[p];
}

__global__ void k_bc_offsets(const i64* __restrict__ toff, const i64* __restrict__ pos, i64 n,
                             i64* __restrict__ offsets, i64* __restrict__ nnz, const u32* __restrict__ err) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += (i64)gridDim.x * blockDim.x) {
        offsets[r] = pos[toff[r]];
        if (r == n) *nnz = (*err) ? (i64)-1 : pos[toff[n]];
    }
}

struct BuildWs {
    i32* cnt;
    i32* cursor;
    i64* toff;
    i32* tidx;
    i32* keep;
    i64* pos;
    i64* partials;
    u32* err;
    SegSortWs sort;
};

static BuildWs carve_build(Carver& c, i64 n, i64 E) {
    BuildWs w;
    const i64 cap = 2 * E;
    w.cnt = c.take<i32>(n + 1);
    w.cursor = c.take<i32>(n + 1);
    w.toff = c.take<i64>(n + 1);
    w.tidx = c.take<i32>(cap);
    w.keep = c.take<i32>(cap);
    w.pos = c.take<i64>(cap + 1);
    w.partials = c.take<i64>(scan_partials_size(std::max(n + 1, cap + 1)));
    w.err = c.take<u32>(4);
    w.sort.tmp = c.take<i32>(cap);
    w.sort.lists = c.take<i32>(3 * (n + 1));
    w.sort.counters = c.take<u32>(4);
    return w;
}

static int bits_for(i64 maxval) {
    int b = 0;
    while (b < 31 && (((i64)1 << b) <= maxval)) ++b;
    return b;
}

}  // namespace fglt

using namespace fglt;

extern "C" size_t fglt_build_csr_workspace(int64_t n, int64_t num_edges) {
    if (n < 0 || num_edges < 0) return 0;
    Carver c(nullptr, 0);
    carve_build(c, n, num_edges);
    return c.used;
}

extern "C" int fglt_build_csr(int64_t n, int64_t num_edges, const int32_t* src, const int32_t* dst,
                              int64_t* offsets, int32_t* indices, int64_t* nnz, void* ws, size_t ws_bytes,
                              void* stream) {
    if (n < 0 || n >= ((int64_t)1 << 31) || num_edges < 0 || num_edges >= ((int64_t)1 << 31)) return FGLT_EINVAL;
    if (!offsets || !nnz || (num_edges > 0 && (!src || !dst || !indices))) return FGLT_EINVAL;
    if (!ws) return FGLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    BuildWs w = carve_build(c, n, num_edges);
    if (!c.ok()) return FGLT_EWORKSPACE;
    const i64 E = num_edges;
    const i64 cap = 2 * E;
    FGLT_HIP_TRY(fill_u32(w.cnt, n + 1, 0u, s));
    FGLT_HIP_TRY(fill_u32(w.cursor, n + 1, 0u, s));
    FGLT_HIP_TRY(fill_u32(w.err, 4, 0u, s));
    const unsigned ge = (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(E, 256), 65536));
    if (E > 0) hipLaunchKernelGGL(k_bc_count, dim3(ge), dim3(256), 0, s, src, dst, E, n, w.cnt, w.err);
    FGLT_LAUNCH_CHECK();
    FGLT_HIP_TRY(scan_exclusive_i32_to_i64(w.cnt, w.toff, n, w.partials, s));
    if (E > 0)
        hipLaunchKernelGGL(k_bc_scatter, dim3(ge), dim3(256), 0, s, src, dst, E, n, w.toff, w.cursor, w.tidx);
    FGLT_LAUNCH_CHECK();
    if (n > 0 && E > 0) {
        FGLT_HIP_TRY(seg_sort(w.tidx, w.toff, n, bits_for(n - 1), w.sort, 65536, s));
        const unsigned gp = (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(cap, 256), 65536));
        hipLaunchKernelGGL(k_bc_keep, dim3(gp), dim3(256), 0, s, w.tidx, w.toff, n, w.keep);
        hipLaunchKernelGGL(k_bc_rowstart, dim3((unsigned)std::min<i64>(ceil_div(n, 256), 65536)), dim3(256), 0, s,
                           w.toff, n, w.keep);
        FGLT_LAUNCH_CHECK();
    }
    // Entries in [toff[n], cap) are never written by the scatter (duplicates
    // and self-loops were skipped); clear their flags so the scan total is exact.
    if (cap > 0) {
        const unsigned gp = (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(cap, 256), 65536));
        hipLaunchKernelGGL(k_bc_zero_tail, dim3(gp), dim3(256), 0, s, w.keep, w.toff, n, cap);
        FGLT_LAUNCH_CHECK();
    }
    FGLT_HIP_TRY(scan_exclusive_i32_to_i64(w.keep, w.pos, cap, w.partials, s));
    if (cap > 0) {
        const unsigned gp = (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(cap, 256), 65536));
        hipLaunchKernelGGL(k_bc_compact, dim3(gp), dim3(256), 0, s, w.tidx, w.keep, w.pos, w.toff, n, indices);
    }
    hipLaunchKernelGGL(k_bc_offsets, dim3((unsigned)std::max<i64>(1, std::min<i64>(ceil_div(n + 1, 256), 65536))),
                       dim3(256), 0, s, w.toff, w.pos, n, offsets, nnz, w.err);
    FGLT_LAUNCH_CHECK();
    return FGLT_OK;
}
