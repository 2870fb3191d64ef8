// raw_prep.hip -- input checks, degree ranking, relabelled CSR and the
// per-entry work counts that drive the counting passes.
#include <algorithm>

#include "walk.h"

namespace fglt {

static constexpr int PT = 256;  // threads per block for the simple kernels


static int bits_for(i64 maxval) {
    int b = 0;
    while (b < 31 && (((i64)1 << b) <= maxval)) ++b;
    return b;
}

// ------------------------------------------------------------ input checks

__global__ void __launch_bounds__(PT) k_check_offsets(const i64* __restrict__ off, i64 n, i64 nnz, i32* __restrict__ deg,
                                DevPlan* plan) {
    i64 dmax = 0;
    u32 err = 0;
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        const i64 a = off[r], b = off[r + 1];
        i64 d = b - a;
        if (d < 0 || a < 0 || b > nnz) {
            err |= ERR_RANGE;
            d = 0;
        }
        if (d >= FGLT_MAX_DEGREE) {
            err |= ERR_DEGREE;
            d = 0;
        }
        deg[r] = (i32)d;
        dmax = d > dmax ? d : dmax;
    }
    if ((i64)blockIdx.x * blockDim.x + threadIdx.x == 0) {
        if (off[0] != 0 || off[n] != nnz) err |= ERR_RANGE;
    }
    __shared__ i64 part[PT / WAVE];
    dmax = block_max<PT>(dmax, part);
    if (threadIdx.x == 0 && dmax > 0) atomicMax((unsigned long long*)&plan->d_max, (unsigned long long)dmax);
    if (err) atomicOr(&plan->err, err);
}

__global__ void k_check_indices(const i32* __restrict__ idx, i64 nnz, i64 n, DevPlan* plan) {
    u32 err = 0;
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (i64)gridDim.x * blockDim.x) {
        const i32 v = idx[p];
        if (v < 0 || (i64)v >= n) err |= ERR_RANGE;
    }
    if (err) atomicOr(&plan->err, err);
}

hipError_t launch_check_input(i64 n, i64 nnz, const i64* off, const i32* idx, RawWs& w, hipStream_t s) {
    static_assert(sizeof(DevPlan) % 4 == 0, "the plan is cleared in 32-bit words");
    hipError_t e = fill_u32(w.plan, sizeof(DevPlan) / 4, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n, PT, 1024)), dim3(PT), 0, s, off, n, nnz, w.deg, w.plan);
    if (nnz > 0) hipLaunchKernelGGL(k_check_indices, dim3(grid_for(nnz, PT, 8192)), dim3(PT), 0, s, idx, nnz, n, w.plan);
    return hipGetLastError();
}

// ------------------------------------------------------------ degree ranking

__global__ void k_rank(const i32* __restrict__ perm, i64 n, i32* __restrict__ rank) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x)
        rank[perm[r]] = (i32)r;
}

// rrow[p] = r for every entry p of row r.  A wavefront takes 4096
// consecutive entries (balanced whatever the row lengths), finds the row of
// its first entry with a 64-way search, then walks 64 entries per step: the
// next 64 row starts (one per lane, strictly increasing past the first row
// with entries) are marked in an LDS row and counted per lane.
static constexpr i64 RF_CHUNK = 4096;
__global__ void __launch_bounds__(PT) k_rowfill(const i64* __restrict__ roff, i64 n, i64 nnz,
                                                i32* __restrict__ rrow) {
    __shared__ i32 flags[PT / WAVE][WAVE];
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    const i64 nw = ((i64)gridDim.x * blockDim.x) / WAVE;
    for (i64 c = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; c * RF_CHUNK < nnz; c += nw) {
        const i64 p0 = c * RF_CHUNK, p1 = std::min<i64>(p0 + RF_CHUNK, nnz);
        // last row r with roff[r] <= p0 (that row has entries, as p0 < nnz)
        i64 lo_ = 0, hi_ = n;
        while (hi_ - lo_ > 1) {
            const i64 step = (hi_ - lo_ + WAVE - 1) / WAVE;
            const i64 q = lo_ + (i64)l * step;
            const int cnt = __popcll(__ballot(q < hi_ && roff[q] <= p0));
            lo_ += (i64)(cnt - 1) * step;
            hi_ = std::min<i64>(hi_, lo_ + step);
        }
        i64 r = lo_;
        for (i64 t0 = p0; t0 < p1; t0 += WAVE) {
            const i64 j = r + 1 + l;
            const i64 stl = j < n ? roff[j] : ((i64)1 << 62);
            const i32 st = stl < t0 + WAVE ? (i32)(stl - t0) : WAVE;  // offset in this step, WAVE when later
            lds_put(&flags[wv][l], 0);
            wave_lds_fence();
            if (st < WAVE) lds_put(&flags[wv][st], 1);
            wave_lds_fence();
            const u64 mask = __ballot(lds_get(&flags[wv][l]) != 0);
            wave_lds_fence();
            const i64 t = t0 + l;
            if (t < p1) rrow[t] = (i32)(r + __popcll(mask & le));
            r += __popcll(mask);
        }
    }
}

// key[q] = rank[idx[off[perm[r]] + (q - roff[r])]] for q in row r of rank
// space: the rows of rank space, each in the caller's column order.
__global__ void __launch_bounds__(PT) k_relabel_copy(const i64* __restrict__ off, const i32* __restrict__ idx,
                                                     const i32* __restrict__ perm, const i32* __restrict__ rank,
                                                     const i64* __restrict__ roff, const i32* __restrict__ rrow,
                                                     i64 nnz, u32* __restrict__ key,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (i64)gridDim.x * blockDim.x) {
        const i64 r = rrow[q];
        const i64 src = off[perm[r]] + (q - roff[r]);
        key[q] = (u32)rank[idx[src]];
    }
}

// Ranks: vertices by (degree, id), a stable radix sort of the pairs
// (degree, id) by degree, which also yields the degrees in rank order.
// Rows: the entries of rank space (r, t) taken row by row are pairs (t, r);
// a stable radix sort by t gathers row t with its columns r in ascending
// order, and the row ids of the sorted pairs are rrow itself.
hipError_t launch_rank_and_relabel(i64 n, i64 nnz, const i64* off, const i32* idx, RawWs& w, hipStream_t s) {
    hipError_t e;
    const i64 nn = std::max<i64>(n, 1);
    // degrees are below min(n, nnz + 1, 2^21) (the checks clamp a larger one to 0)
    const i64 d_bound = std::min<i64>({n - 1, nnz, FGLT_MAX_DEGREE - 1});
    // pass buffers: ek holds 2 max(nnz, n) and cntd 2 (n + 2) 32-bit words, G 2 (nnz + 1)
    u32* ek_k = reinterpret_cast<u32*>(w.ek);
    if ((e = radix_sort_pairs(n, bits_for(d_bound), reinterpret_cast<const u32*>(w.deg), nullptr,
                              reinterpret_cast<u32*>(w.rdeg), w.perm, ek_k, reinterpret_cast<i32*>(ek_k + nn),
                              reinterpret_cast<u32*>(w.cntd), reinterpret_cast<i32*>(w.cntd) + nn, w.rx_hist,
                              w.partials, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, w.perm, n, w.rank);
    if ((e = scan_exclusive_i32_to_i64(w.rdeg, w.roff, n, w.partials, s)) != hipSuccess) return e;
    if (nnz > 0) {
        hipLaunchKernelGGL(k_rowfill, dim3(grid_for(nnz, PT / WAVE * RF_CHUNK, 65536)), dim3(PT), 0, s, w.roff, n,
                           nnz, w.rrow);
        u32* g_k = reinterpret_cast<u32*>(w.G);
        hipLaunchKernelGGL(k_relabel_copy, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, off, idx, w.perm, w.rank,
                           w.roff, w.rrow, nnz, g_k, (const u32*)&w.plan->err);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // pass 1 reads (G, rrow); later passes alternate between ek and G
        if ((e = radix_sort_pairs(nnz, bits_for(n - 1), g_k, w.rrow, nullptr, w.ridx, ek_k,
                                  reinterpret_cast<i32*>(ek_k + nnz), g_k, reinterpret_cast<i32*>(g_k + nnz),
                                  w.rx_hist, w.partials, s)) != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ structure

// lo[u] = |N-(u)| (entries < u); self-loop check; sum of lo; the number of
// vertices of degree <= 1.
__global__ void __launch_bounds__(PT) k_lo(const i64* __restrict__ roff, const i32* __restrict__ ridx, i64 n,
                                           i32* __restrict__ lo, VRec* __restrict__ vrec, DevPlan* plan) {
    FGLT_GATE(&plan->err);
    __shared__ i64 part[PT / WAVE];
    i64 sum = 0, low = 0;
    u32 err = 0;
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (i64)gridDim.x * blockDim.x) {
        const i64 b = roff[u], e = roff[u + 1];
        const i64 q = lower_bound_dev(ridx, b, e, (i32)u);
        if (q < e && ridx[q] == (i32)u) err |= ERR_SELFLOOP;
        lo[u] = (i32)(q - b);
        vrec[u] = VRec{b, (i32)(q - b), (i32)(e - b)};
        sum += q - b;
        low += e - b <= 1;
    }
    sum = block_sum<PT>(sum, part);
    if (threadIdx.x == 0 && sum) atomicAdd((unsigned long long*)&plan->sum_lo, (unsigned long long)sum);
    low = block_sum<PT>(low, part);
    if (threadIdx.x == 0 && low) atomicAdd((unsigned long long*)&plan->n_low, (unsigned long long)low);
    if (err) atomicOr(&plan->err, err);
}

// rpos / mirror / work count per entry; duplicate and symmetry checks.
//   N- entry (u, v), v < u: rpos = position of u in row v (= number of
//     neighbours of v below u, the wedge count of the 4-cycle pass); the
//     binary search that finds it gives both mirror positions;
//   N+ entry (v, u), u > v: rpos = -1, work = d+(u) (the triangle pass).
//   A diagonal entry gets rpos = -1 (the input check rejects it).
__global__ void k_rpos(const VRec* __restrict__ vrec, const i32* __restrict__ ridx, const i32* __restrict__ rrow,
                       i64 nnz, i32* __restrict__ rpos, i64* __restrict__ mir, i64* __restrict__ G,
                       int with_c4, DevPlan* plan) {
    FGLT_GATE(&plan->err);
    u32 err = 0;
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (i64)gridDim.x * blockDim.x) {
        {
            const i64 u = rrow[p];
            const i32 v = ridx[p];
            if (p > 0 && rrow[p - 1] == (i32)u && ridx[p - 1] == v) err |= ERR_DUP;
            const VRec rv = vrec[v];  // one 16-byte load: start, |N-(v)|, degree
            i64 work = 0;
            if ((i64)v < u) {
                const i64 b = rv.off + rv.lo, e = rv.off + rv.deg;
                const i64 q = lower_bound_dev(ridx, b, e, (i32)u);
                i32 rp = 0;  // on an asymmetric input: harmless, no wedges (the run stops there)
                if (q < e && ridx[q] == (i32)u) {
                    rp = (i32)(q - rv.off);
                    mir[p] = q;
                    mir[q] = p;  // the mirror (v, u) learns where (u, v) sits
                } else {
                    err |= ERR_ASYM;
                    mir[p] = p;  // harmless: the run stops at the input check
                }
                rpos[p] = rp;
                work = with_c4 ? rp : 0;  // no 4-cycle pass: no wedge work, no 4-cycle tiers
            } else {
                if ((i64)v > u) work = rv.deg - rv.lo;  // mir[p] comes from the mirror's thread
                rpos[p] = -1;
            }
            G[p] = work;
        }
    }
    if (err) atomicOr(&plan->err, err);
}

// Appends the threads of class cls >= 0 to lists[cls * n + ...]: one ballot
// per class and wavefront, one global atomic per class and workgroup.
template <int NT, int K>
__device__ __forceinline__ void block_append(int cls, i32 value, u32* __restrict__ counters, i32* __restrict__ lists,
                                             i64 n, u32 (*wcnt)[K], u32* sbase) {
    const int wv = threadIdx.x / WAVE, l = lane_id();
    u32 rank = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const u64 m = __ballot(cls == c);
        if (l == 0) wcnt[wv][c] = (u32)__popcll(m);
        if (cls == c) rank = (u32)__popcll(m & lanemask_lt());
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
        const int c = threadIdx.x;
        u32 run = 0;
        for (int w = 0; w < NT / WAVE; ++w) {
            const u32 x = wcnt[w][c];
            wcnt[w][c] = run;
            run += x;
        }
        sbase[c] = run ? atomicAdd(&counters[c], run) : 0;
    }
    __syncthreads();
    if (cls >= 0) lists[(i64)cls * n + sbase[cls] + wcnt[wv][cls] + rank] = value;
    __syncthreads();
}

// Tier lists and statistics from the work counts (G holds the exclusive scan).
static constexpr int TT = 1024;
__global__ void __launch_bounds__(TT) k_tiers(const i64* __restrict__ roff, const i32* __restrict__ lo,
                                              const i32* __restrict__ rdeg, const i64* __restrict__ G, i64 n,
                                              Tiers th, i32* __restrict__ tri_list, i32* __restrict__ c4_list,
                                              DevPlan* plan) {
    FGLT_GATE(&plan->err);
    __shared__ u32 wt[TT / WAVE][3], wc[TT / WAVE][4];
    __shared__ u32 bt[3], bc[4];
    __shared__ i64 part[TT / WAVE];
    i64 dpmax = 0;
    i64 titems[3] = {0, 0, 0}, witems[4] = {0, 0, 0, 0};
    i64 etab = 0;  // window tier: |N-(u)| x (windows + 1) entries of the per-entry window table
    i64 heavy = 0; // window-tier vertices of degree >= 65536
    for (i64 u0 = (i64)blockIdx.x * TT; u0 < n; u0 += (i64)gridDim.x * TT) {
        const i64 u = u0 + threadIdx.x;
        int tcls = -1, ccls = -1;
        if (u < n) {
            const i64 b = roff[u], m = roff[u] + lo[u], e = roff[u + 1];
            const i64 D = e - m;
            const i64 W = G[m] - G[b];
            const i64 T = G[e] - G[m];
            dpmax = D > dpmax ? D : dpmax;
            if (D >= 2) tcls = D <= th.tri_wave ? 0 : (D <= th.tri_lds ? 1 : 2);
            if (W > 0) {
                const i64 L = m - b;
                ccls = W <= th.c4_wave ? 0
                       : W <= th.c4_block ? 1
                       : (W <= th.c4_hash && L <= th.c4_hash_lmax) ? 2 : 3;
            }
            if (tcls >= 0) titems[tcls] += T;
            if (ccls >= 0) witems[ccls] += W;
            if (ccls == 3) {
                if (e - b < 65536) etab += (m - b) * ((u + C4W_SPAN - 1) / C4W_SPAN + 1);
                else ++heavy;
            }
        }
        block_append<TT, 3>(tcls, (i32)u, plan->n_tri, tri_list, n, wt, bt);
        block_append<TT, 4>(ccls, (i32)u, plan->n_c4, c4_list, n, wc, bc);
    }
    dpmax = block_max<TT>(dpmax, part);
    if (threadIdx.x == 0 && dpmax > 0) atomicMax((unsigned long long*)&plan->dplus_max, (unsigned long long)dpmax);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const i64 ti = block_sum<TT>(titems[c], part);
        if (threadIdx.x == 0 && ti) atomicAdd((unsigned long long*)&plan->tri_items_tier[c], (unsigned long long)ti);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const i64 wi = block_sum<TT>(witems[c], part);
        if (threadIdx.x == 0 && wi) atomicAdd((unsigned long long*)&plan->wedge_items_tier[c], (unsigned long long)wi);
    }
    etab = block_sum<TT>(etab, part);
    if (threadIdx.x == 0 && etab) atomicAdd((unsigned long long*)&plan->c4_etab, (unsigned long long)etab);
    heavy = block_sum<TT>(heavy, part);
    if (threadIdx.x == 0 && heavy) atomicAdd(&plan->n_c4_heavy, (u32)heavy);
}

__global__ void __launch_bounds__(PT) k_totals(const i64* __restrict__ roff, const i32* __restrict__ lo,
                                               const i64* __restrict__ G, i64 n, i64 nnz, DevPlan* plan) {
    FGLT_GATE(&plan->err);
    __shared__ i64 part[PT / WAVE];
    i64 wedges = 0;
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (i64)gridDim.x * blockDim.x)
        wedges += G[roff[u] + lo[u]] - G[roff[u]];
    wedges = block_sum<PT>(wedges, part);
    if (threadIdx.x == 0 && wedges) atomicAdd((unsigned long long*)&plan->wedge_items, (unsigned long long)wedges);
}

int bits_for_n(i64 n) {
    int b = 0;
    while (b < 31 && (((i64)1 << b) <= n - 1)) ++b;
    return b;
}

Tiers tiers_from_plan(const fglt_raw_plan* plan, i64 n) {
    Tiers t{TRI_WAVE_MAX, TRI_LDS_MAX, TRI_HUB_MAX, C4_WAVE_MAX, C4_BLOCK_MAX, C4_HASH_MAX, 0, 0, 0};
    if (plan) {
        if (plan->tri_wave_max > 0) t.tri_wave = std::min<i64>(plan->tri_wave_max, TRI_WAVE_MAX);
        if (plan->tri_lds_max > 0) t.tri_lds = std::min<i64>(plan->tri_lds_max, TRI_LDS_MAX);
        if (plan->tri_hub_max > 0) t.tri_hub = std::min<i64>(plan->tri_hub_max, TRI_HUB_MAX);
        if (plan->tri_hub_max < 0) t.tri_hub = 0;
        if (plan->c4_wave_max > 0) t.c4_wave = std::min<i64>(plan->c4_wave_max, C4_WAVE_MAX);
        if (plan->c4_wave_max < 0) t.c4_wave = 0;
        if (plan->c4_block_max > 0) t.c4_block = std::min<i64>(plan->c4_block_max, C4_BLOCK_MAX);
        if (plan->c4_block_max < 0) t.c4_block = 0;
        if (plan->c4_hash_max > 0) t.c4_hash = std::min<i64>(plan->c4_hash_max, C4_HASH_MAX);
        if (plan->c4_hash_max < 0) t.c4_hash = 0;
        if (plan->c4_window_rows == 1 || plan->c4_window_rows == 2) t.c4_rows = plan->c4_window_rows;
        if (plan->c4_window_group > 0) t.c4_group = std::min<int>(plan->c4_window_group, 1024);
    }
    t.tri_lds = std::max(t.tri_lds, t.tri_wave);
    t.c4_block = std::max(t.c4_block, t.c4_wave);
    t.c4_hash = std::max(t.c4_hash, t.c4_block);
    // a hash word holds the rank of a wedge end in the high bits and its count
    // (at most |N-(u)|) in the remaining low bits
    const int kb = std::max(1, bits_for_n(n));
    t.c4_hash_lmax = ((i64)1 << (32 - kb)) - 1;
    return t;
}

// Every entry below the diagonal has its mirror (k_rpos) and half the entries
// lie below it: the CSR is symmetric.  One thread.
__global__ void k_check_half(DevPlan* plan, i64 nnz) {
    if (2 * plan->sum_lo != nnz) atomicOr(&plan->err, ERR_ASYM);
}

// What the host no longer waits for: whether the bitmaps of the wave, LDS and
// hub tiers fit the workspace (the clique pass then reads them), and whether
// the window tier's per-entry table does.  One thread.
__global__ void k_plan_decide(DevPlan* plan, const i64* __restrict__ bitmap_words, i64 bstore_cap, int want_store,
                              int want_etab) {
    plan->stored = want_store && !plan->err && *bitmap_words <= bstore_cap;
    plan->use_etab = want_etab && !plan->err && plan->c4_etab <= 4 * bstore_cap;
}

hipError_t launch_structure(i64 n, i64 nnz, RawWs& w, const Tiers& th, bool with_c4, bool want_store, int rows_mode,
                            hipStream_t s) {
    hipError_t e;
    hipLaunchKernelGGL(k_lo, dim3(grid_for(n, PT, 1024)), dim3(PT), 0, s, w.roff, w.ridx, n, w.lo, w.vrec, w.plan);
    hipLaunchKernelGGL(k_check_half, dim3(1), dim3(1), 0, s, w.plan, nnz);
    if (nnz > 0)
        hipLaunchKernelGGL(k_rpos, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, w.vrec, w.ridx, w.rrow, nnz,
                           w.rpos, w.mir, w.G, with_c4 ? 1 : 0, w.plan);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_exclusive_i64(w.G, w.G, nnz, w.partials, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tiers, dim3(grid_for(n, TT, 256)), dim3(TT), 0, s, w.roff, w.lo, w.rdeg, w.G, n, th,
                       w.tri_list, w.c4_list, w.plan);
    hipLaunchKernelGGL(k_totals, dim3(grid_for(n, PT, 1024)), dim3(PT), 0, s, w.roff, w.lo, w.G, n, nnz, w.plan);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // bitmap rows of the wave, LDS and hub tiers (the clique pass reads them)
    if ((e = launch_bitmap_offsets(n, w, std::max(th.tri_lds, th.tri_hub), s)) != hipSuccess) return e;
    // the per-entry window table needs the 16-bit vertex table (its capacity is known here)
    const i64 k1 = (n + C4W_SPAN - 1) / C4W_SPAN + 1, ts = (k1 + 15) & ~(i64)15;
    const bool want_etab = rows_mode == 0 && w.c4_tab != nullptr && n * ts <= w.c4_tab_cap;
    hipLaunchKernelGGL(k_plan_decide, dim3(1), dim3(1), 0, s, w.plan, (const i64*)(w.boff + n), w.bstore_cap,
                       want_store ? 1 : 0, want_etab ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------ workspace layout

RawWs carve_raw(Carver& c, i64 n, i64 nnz) {
    RawWs w{};
    const i64 nn = std::max<i64>(n, 1);
    w.plan = c.take<DevPlan>(1);
    w.deg = c.take<i32>(nn);
    w.perm = c.take<i32>(nn);
    w.rank = c.take<i32>(nn);
    w.rdeg = c.take<i32>(nn);
    w.lo = c.take<i32>(nn);
    w.cntd = c.take<i64>(nn + 2);
    w.roff = c.take<i64>(nn + 1);
    w.vrec = c.take<VRec>(nn);
    w.l2rec = c.take<L2Rec>(nn);
    w.ridx = c.take<i32>(nnz);
    w.rpos = c.take<i32>(nnz);
    w.mir = c.take<i64>(nnz);
    w.rrow = c.take<i32>(nnz);
    w.G = c.take<i64>(nnz + 1);
    w.C3 = c.take<i32>(nnz);
    w.acc = c.take<i64>(10 * nn);
    if (w.acc) {
        w.sumd = w.acc + 0 * nn;
        w.s7 = w.acc + 1 * nn;
        w.c3x2 = w.acc + 2 * nn;
        w.ap2 = w.acc + 3 * nn;
        w.ac3 = w.acc + 4 * nn;
        w.d10 = w.acc + 5 * nn;
        w.d14 = w.acc + 6 * nn;
        w.d13 = w.acc + 7 * nn;
        w.c4v = w.acc + 8 * nn;
        w.k4v = w.acc + 9 * nn;
    }
    w.tri_list = c.take<i32>(3 * nn);
    w.c4_list = c.take<i32>(4 * nn);
    // out-degree under the degree ordering is at most sqrt(nnz): two bitmaps
    // of D x ceil(D/64) words fit in tri_slot_words.  The clique pass above
    // the hub tier has as many slots of that size as fit max(1 GiB, 2 bytes
    // per entry), from 1 to 64 (its launch for out-degrees up to TRI_MID_D
    // cuts the same memory into smaller slots).
    i64 dmax_plus = 1;
    while (dmax_plus * dmax_plus <= nnz) ++dmax_plus;
    const i64 words_per_row = ceil_div(dmax_plus, 64);
    w.tri_slot_words = 2 * dmax_plus * words_per_row;
    w.tri_nslots = (int)std::max<i64>(
        1, std::min<i64>(NUM_TRI_SLOTS, std::max<i64>((i64)1 << 30, 2 * nnz) / (8 * w.tri_slot_words)));
    w.tri_slots = c.take<u64>(w.tri_nslots * w.tri_slot_words);
    w.tri_jobpre = c.take<i64>(nn + 2);
    w.tri_partials = c.take<i64>(scan_partials_size(nn + 2));
    w.bcnt = c.take<i64>(nn);
    w.boff = c.take<i64>(nn + 1);
    w.c4_segoff = c.take<i64>(2);
    w.c4_jobcnt = c.take<i64>(nn + 1);
    w.c4_jobpre = c.take<i64>(nn + 1);
    w.c4_ebase = c.take<i64>(nn + 1);
    w.c4_hjobcnt = c.take<i64>((nnz >> 16) + 2);
    w.c4_hjobpre = c.take<i64>((nnz >> 16) + 2);
    w.c4_jobctr = c.take<u32>(4);
    // vertex window table: n x (ceil(n / 65536) + 1) 16-bit entries, rows
    // padded to 16 entries, when that stays within max(1 GiB, 8 bytes per entry)
    {
        const i64 k1 = ((nn + C4W_SPAN - 1) / C4W_SPAN + 1 + 15) & ~(i64)15;
        const i64 entries = nn * k1;
        w.c4_tab_cap = entries * 2 <= std::max<i64>((i64)1 << 30, 8 * nnz) ? entries : 0;
        w.c4_tab = w.c4_tab_cap ? c.take<u16>(w.c4_tab_cap) : nullptr;
        if (!c.base) w.c4_tab = nullptr;
    }
    // window-tier scratch: up to 2^20 words per workgroup, at most nnz / 16
    // a multiple of 64 words, so that every workgroup's slice starts on a
    // 256-byte boundary (the pass C stream reads it 16 bytes at a time)
    w.c4_scr_cap = std::max<i64>(std::min<i64>((i64)1 << 20, nnz / 16), 1024) & ~(i64)63;
    w.c4_scr = c.take<u32>(C4W_GRID * w.c4_scr_cap);
    w.partials = c.take<i64>(scan_partials_size(std::max(nn + 2, nnz + 1)));
    w.ek = c.take<i64>(std::max(nnz, nn));
    w.sort.tmp = reinterpret_cast<i32*>(w.ek);  // dead once the relabelled rows are built
    w.sort.lists = c.take<i32>(3 * (nn + 2));
    w.sort.counters = c.take<u32>(4);
    w.rx_hist = c.take<i64>(radix_hist_size(std::max(nnz, nn)));
    // the stored bitmaps last: at least 3 words per entry (1 beyond 2^31
    // entries), and whatever a larger workspace holds beyond the rest (the
    // clique pass reads stored bitmaps only when all of them fit).  The
    // window tier's per-entry table reuses this memory: when the vertex table
    // is there and a bound on the per-entry table, (nnz / 2) (n / 65536 + 2)
    // 16-bit entries, stays within 80 bytes per entry, the memory holds it.
    {
        i64 min_words = std::max<i64>(nnz < ((i64)1 << 31) ? 3 * nnz : nnz, 64);
        const i64 etab_bound = (nnz / 2) * ((nn + C4W_SPAN - 1) / C4W_SPAN + 2);
        if (w.c4_tab_cap && 2 * etab_bound <= 80 * nnz) min_words = std::max(min_words, ceil_div(etab_bound, 4));
        i64 words = min_words;
        if (c.base && c.cap > c.used + 512) words = std::max<i64>(min_words, (i64)((c.cap - c.used - 512) / 8));
        w.bstore_cap = words;
        w.bstore = c.take<u64>(words);
    }
    return w;
}

}  // namespace fglt
