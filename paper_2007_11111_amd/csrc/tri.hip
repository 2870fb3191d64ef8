// tri.hip -- triangle pass with stored neighbourhood bitmaps, and the clique /
// diamond pass that reuses them.
//
// Triangle pass (per vertex u with out-degree D = |N+(u)|, N+(u) in LDS):
//   the out-lists N+(v) of every v in N+(u) are walked as one flattened item
//   stream (coalesced, 64 consecutive items per wavefront step); each item y
//   is looked up in an LDS position map of N+(u).  A hit at position l is a
//   triangle (u, v_k, v_l): bit l of row k of the bitmap B (the induced
//   subgraph H on N+(u)) is set, and C3 of (v_k, v_l) counted by one global
//   atomic; C3 of the edges (u, v_k) follows from B's rows and columns.  B is
//   stored for the clique pass when the workspace holds it.  The wave tier
//   packs several small vertices into one wavefront.
// Clique / diamond pass from stored bitmaps: B is reloaded and A = B | B^T
//   formed; every edge (k, l) of H lies on |A_k & A_l| triangles of H, each a
//   4-clique with u, so every 4-clique {u < a < b < c} and every off-cord
//   diamond of a triangle with lowest vertex u is attributed to its vertices
//   (Section IV-C: T e / 6 and D4,c e / 2 without forming T or D4,c).  The
//   diamond term of u needs C3 of the edge (v_k, v_l): a galloping search of
//   v_l in N+(v_k) in the wave tier, a second walk of the out-lists in the LDS
//   tier.  The counts of the N+ vertices are stored at the mirrored entries
//   and summed by rows afterwards (no per-entry atomics).
#include <algorithm>

#include "walk.h"

namespace fglt {

static constexpr int WT = 256;  // wave-tier block: 4 independent wavefronts
static constexpr int LT = 512;  // LDS-tier block: 8 wavefronts on one vertex

// ------------------------------------------------------------------ triangle pass

// C3 of the edge (v_k, v_l) of a triangle is a global counter.  A device-scope
// atomic issued between the gathers of a walk holds back the next gather
// (vector memory operations complete in order), so the walk queues the entry
// indices of its hits in LDS -- one ballot per step, no LDS atomic -- and the
// wavefront issues the increments after the walk.  A full queue (or entry
// indices beyond 32 bits: defer == 0) falls back to the direct atomic.
static constexpr int TRI_QCAP = 512;

__device__ __forceinline__ void defer_c3(bool hit, i64 e, u32* q, u32& nq, i32* __restrict__ C3, int defer) {
    const u64 hm = __ballot(hit);
    if (!hm) return;
    const u32 pos = nq + (u32)__popcll(hm & lanemask_lt());
    if (hit) {
        if (defer && pos < TRI_QCAP) q[pos] = (u32)e;
        else atomicAdd(&C3[e], 1);
    }
    nq += (u32)__popcll(hm);
}

__device__ __forceinline__ void flush_c3(const u32* q, u32 nq, i32* __restrict__ C3, int lane, int width) {
    const u32 cnt = nq < (u32)TRI_QCAP ? nq : (u32)TRI_QCAP;
    for (u32 i = lane; i < cnt; i += width) atomicAdd(&C3[q[i]], 1);
}

// Wave tier of the triangle pass.  A wavefront takes TASK consecutive
// vertices of the tier list at a time and packs consecutive ones whose
// out-degrees sum to at most 64 into one round: vertex g's out-neighbours on
// lanes off_g + k, one shared position map keyed by (v, g) (v | g << 28, so
// PACK needs n <= 2^28), the out-lists of all of them walked as one item
// stream, and bitmap bits at the lanes' positions (the 64 x 64 transpose then
// transposes every vertex's block on its own).  Tasks come from the end of
// the list first, where the vertices of high out-degree sit.
template <bool PACK>
__global__ void __launch_bounds__(WT) k_tri1_wave(const VRec* __restrict__ vrec, const i32* __restrict__ ridx,
                                                  const i32* __restrict__ list, const u32* __restrict__ countp, i32* __restrict__ C3,
                                                  u64* __restrict__ bstore, const i64* __restrict__ boff, const u32* __restrict__ storep,
                                                  int defer) {
    const int store = (int)*storep;  // the bitmaps are stored (decided on the device)
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int NW = WT / WAVE;
    constexpr int TASK = PACK ? 8 : 1;
    __shared__ i64 rbase[NW][WAVE + 1];
    __shared__ i32 rstart[NW][WAVE + 1];
    __shared__ i32 rk[NW][WAVE + 1];  // lane of run r, with its vertex slot above bit 8
    __shared__ BucketMap<6> pm[NW];   // positions of the round's out-neighbours: 64 buckets of 4
    __shared__ i32 flags[NW][WAVE];
    __shared__ u64 sB[NW][WAVE];
    __shared__ u32 sQ[NW][TRI_QCAP];  // deferred C3 increments (entry indices)
    const int wid = threadIdx.x / WAVE;
    const int lane = lane_id();
    const u64 le = lane == WAVE - 1 ? ~0ull : ((1ull << (lane + 1)) - 1);
    auto key = [](i32 v, i32 g) { return PACK ? (v | (g << 28)) : v; };
    // every wavefront runs its own vertices; it shares no LDS with the others,
    // so only wavefront-level fences order its steps
    const i64 ntasks = ((i64)count + TASK - 1) / TASK;
    for (i64 tj = (i64)blockIdx.x * NW + wid; tj < ntasks; tj += (i64)gridDim.x * NW) {
        const i64 t0 = (ntasks - 1 - tj) * TASK;
        const int ntask = (int)std::min<i64>(TASK, (i64)count - t0);
        i64 u_i = 0, bu_i = 0, bo_i = 0;
        i32 D_i = 0;
        if (lane < ntask) {
            u_i = list[t0 + lane];
            const VRec r = vrec[u_i];
            bu_i = r.off + r.lo;
            D_i = r.deg - r.lo;
            bo_i = boff[u_i];
        }
        for (int next = 0; next < ntask;) {
            // this round: vertices next .. next + P - 1 (out-degrees sum to at most 64)
            const i32 dd = (lane >= next && lane < ntask) ? D_i : 0;
            const i32 incl = wave_incl_scan_i32(dd);
            const u64 inr = __ballot(lane >= next && lane < ntask && incl <= WAVE);
            const int P = __popcll(inr);
            const i32 excl = incl - dd;
            bmap_clear(pm[wid], lane, WAVE);
            sB[wid][lane] = 0;
            lds_put(&flags[wid][lane], 0);
            wave_lds_fence();
            if ((inr >> lane) & 1ull) lds_put(&flags[wid][excl], 1);
            wave_lds_fence();
            const u64 starts = __ballot(lds_get(&flags[wid][lane]) != 0);
            wave_lds_fence();
            const i32 used = __builtin_amdgcn_readlane(incl, next + P - 1);
            const int gl = __popcll(starts & le) - 1;  // vertex slot of this lane in the round
            const int g = next + gl;
            const bool act = lane < used;
            const i64 bu = __shfl(bu_i, g, WAVE);
            const i64 bo = __shfl(bo_i, g, WAVE);
            const i32 off_g = __shfl(excl, g, WAVE);
            const i32 k = lane - off_g;
            i32 len = 0;
            i64 bv = 0;
            if (act) {
                const i32 v = ridx[bu + k];
                bmap_insert(pm[wid], key(v, gl), lane);
                const VRec rv = vrec[v];
                bv = rv.off + rv.lo;
                len = rv.deg - rv.lo;  // |N+(v)|: the items of this run
            }
            const i32 iincl = wave_incl_scan_i32(len);
            const i32 pre = iincl - len;
            const i32 T = __builtin_amdgcn_readlane(iincl, WAVE - 1);
            const u64 m = __ballot(len > 0);
            const i32 nruns = __popcll(m);
            if (len > 0) {
                const int c = __popcll(m & lanemask_lt());
                rbase[wid][c] = bv - pre;
                rstart[wid][c] = pre;
                rk[wid][c] = lane | (gl << 8);
            }
            if (lane == 0) rstart[wid][nruns] = T;
            wave_lds_fence();
            u32 nq = 0;  // wave-uniform
            if (T > 0) {
                run_walk_keyed<4>(0, T, rbase[wid], rstart[wid], rk[wid], nruns, flags[wid], ridx,
                                  [&](bool a, i32, i32 rkey, i32 y, i64 e, u64, i32) {
                    const i32 kr = a ? rkey : 0;
                    const i32 l = a ? bmap_find(pm[wid], key(y, kr >> 8)) : -1;
                    const bool hit = l >= 0;
                    if (hit) atomicOr((unsigned long long*)&sB[wid][kr & 0xff], 1ull << l);
                    defer_c3(hit, e, sQ[wid], nq, C3, defer);
                });
            }
            wave_lds_fence();
            flush_c3(sQ[wid], nq, C3, lane, WAVE);
            // triangles on the edge (u, v_k): row k of B (v_l in N+(v_k)) plus
            // column k (v_k in N+(v_j)) of the induced subgraph on N+(u)
            const u64 row = sB[wid][lane];
            const u64 col = wave_transpose64(row);
            if (act) {
                const i32 c = __popcll(row) + __popcll(col);
                if (c) atomicAdd(&C3[bu + k], c);
                if (store) bstore[bo + k] = row >> off_g;
            }
            wave_lds_fence();  // the next round clears the map and the rows
            next += P;
        }
    }
}

__global__ void __launch_bounds__(LT) k_tri1_lds(const i64* __restrict__ roff, const VRec* __restrict__ vrec, const i32* __restrict__ ridx,
                                                 const i32* __restrict__ lo, const i64* __restrict__ G,
                                                 const i32* __restrict__ list, const u32* __restrict__ countp, i32* __restrict__ C3,
                                                 u64* __restrict__ bstore, const i64* __restrict__ boff, const u32* __restrict__ storep,
                                                 int defer) {
    const int store = (int)*storep;  // the bitmaps are stored (decided on the device)
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int DM = TRI_LDS_MAX;
    constexpr int WM = DM / 64;
    constexpr int NWV = LT / WAVE;
    __shared__ i64 rbase[DM + 1];
    __shared__ i32 rstart[DM + 1];
    __shared__ i32 rk[DM + 1];
    __shared__ BucketMap<9> pm;  // positions of N+(u): 512 buckets of 4
    __shared__ i32 flags[NWV][WAVE];
    __shared__ i32 Cnt[DM];
    __shared__ u64 B[DM * WM];
    __shared__ i32 wsum[NWV];
    __shared__ i32 stot, sR;
    __shared__ u32 sQ[NWV][TRI_QCAP];  // deferred C3 increments per wavefront
    const int wv = threadIdx.x / WAVE;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        const int W = (D + 63) >> 6;
        const i64 gb = G[bu];
        const i32 T = (i32)(G[bu + D] - gb);
        bmap_clear(pm, threadIdx.x, LT);
        for (int q = threadIdx.x; q < D * W; q += LT) B[q] = 0;
        __syncthreads();
        const int k = threadIdx.x;  // D <= DM == LT: one out-neighbour per thread
        i32 len = 0, pre = 0;
        i64 bv = 0;
        if (k < D) {
            const i32 v = ridx[bu + k];
            bmap_insert(pm, v, k);
            pre = (i32)(G[bu + k] - gb);
            len = (i32)(G[bu + k + 1] - G[bu + k]);
            { const VRec rv = vrec[v]; bv = rv.off + rv.lo; }
        }
        const i32 cidx = block_scan<LT>(len > 0 ? 1 : 0, wsum, &stot);
        if (k < D && len > 0) {
            rbase[cidx] = bv - pre;
            rstart[cidx] = pre;
            rk[cidx] = k;
        }
        if (threadIdx.x == 0) {
            sR = stot;
            rstart[stot] = T;
        }
        __syncthreads();
        const i32 per = ((T + NWV * WAVE - 1) / (NWV * WAVE)) * WAVE;
        u32 nq = 0;  // wave-uniform
        run_walk_keyed<4>(std::min(T, wv * per), std::min(T, (wv + 1) * per), rbase, rstart, rk, sR, flags[wv], ridx,
                          [&](bool act, i32, i32 kr, i32 y, i64 e, u64, i32) {
                        const i32 l = act ? bmap_find(pm, y) : -1;
                        const bool hit = l >= 0;
                        if (hit) atomicOr((unsigned long long*)&B[kr * W + (l >> 6)], 1ull << (l & 63));
                        defer_c3(hit, e, sQ[wv], nq, C3, defer);
                    });
        __syncthreads();
        flush_c3(sQ[wv], nq, C3, lane_id(), WAVE);
        // C3 of the edge (u, v_k): the triangles in row k of B plus those in
        // column k, counted by 64 x 64 block transposes (wavefront bj takes
        // the columns bj * 64 .. bj * 64 + 63, W <= LT / 64)
        if (wv < W) {
            i32 cc = 0;
            for (int bi = 0; bi < W; ++bi) {
                const int row = bi * 64 + lane_id();
                cc += __popcll(wave_transpose64(row < D ? B[row * W + wv] : 0ull));
            }
            Cnt[wv * 64 + lane_id()] = cc;
        }
        __syncthreads();
        if (k < D) {
            i32 c = Cnt[k];
            for (int z = 0; z < W; ++z) c += __popcll(B[k * W + z]);
            if (c) atomicAdd(&C3[bu + k], c);
            if (store)
                for (int z = 0; z < W; ++z) bstore[boff[u] + (i64)k * W + z] = B[k * W + z];
        }
        __syncthreads();
    }
}

// Hub tier of the triangle pass: TRI_LDS_MAX < D <= hub_max (at most
// TRI_HUB_MAX), one vertex per 1024-thread workgroup.  The position map of
// N+(u) and the run arrays stay in LDS; the bitmap B (up to 128 KiB) does not
// fit beside them, so C3 of the edges (u, v_k) is counted in LDS (a hit at
// (k, l) adds one to both), and the hits' bits of B (rows in the workspace,
// read by the clique pass) and C3 increments of the far edges (v_k, v_l) are
// queued per wavefront in LDS and issued in bursts, so that no device-scope
// atomic sits between the walk's gathers.
static constexpr int HT = 1024;        // hub-tier block: 16 wavefronts on one vertex
static constexpr int HUB_QCAP = 256;   // hits queued per wavefront before a burst

// The first rows of B that fit HUB_BWORDS words of LDS are set there (most
// hits: row k holds the bits l > k); the rest go to the workspace rows
// through the queue, marked by HUB_GLOBAL_ROW.
static constexpr int HUB_BWORDS = 9792;         // 576 rows of 17 words
static constexpr u32 HUB_GLOBAL_ROW = 1u << 31;  // queued hit whose bit goes to the workspace row

struct HubQueue {
    u32* qe;   // entry index of the far edge (v_k, v_l)
    u32* qkl;  // k << 16 | l, with HUB_GLOBAL_ROW when row k is not in LDS
    u32 n;     // wave-uniform fill
};

__device__ __forceinline__ void hub_flush(HubQueue& q, i32* __restrict__ C3, u64* __restrict__ Bg, int W) {
    wave_lds_fence();
    for (u32 i = lane_id(); i < q.n; i += WAVE) {
        atomicAdd(&C3[q.qe[i]], 1);
        const u32 kl = q.qkl[i];
        if (Bg && (kl & HUB_GLOBAL_ROW)) {
            const u32 k = (kl >> 16) & 0x7fffu, l = kl & 0xffffu;
            atomicOr((unsigned long long*)&Bg[(i64)k * W + (l >> 6)], 1ull << (l & 63));
        }
    }
    q.n = 0;
    wave_lds_fence();
}

__device__ __forceinline__ void hub_push(bool hit, i64 e, u32 kl, HubQueue& q, i32* __restrict__ C3,
                                         u64* __restrict__ Bg, int W, int defer) {
    const u64 hm = __ballot(hit);
    if (!hm) return;
    if (!defer) {  // entry indices beyond 32 bits: issue at once
        if (hit) {
            atomicAdd(&C3[e], 1);
            if (Bg && (kl & HUB_GLOBAL_ROW))
                atomicOr((unsigned long long*)&Bg[(i64)((kl >> 16) & 0x7fffu) * W + ((kl & 0xffffu) >> 6)],
                         1ull << (kl & 63));
        }
        return;
    }
    const u32 c = (u32)__popcll(hm);
    if (q.n + c > (u32)HUB_QCAP) hub_flush(q, C3, Bg, W);
    if (hit) {
        const u32 pos = q.n + (u32)__popcll(hm & lanemask_lt());
        q.qe[pos] = (u32)e;
        q.qkl[pos] = kl;
    }
    q.n += c;
}

// The out-lists N+(v_k) of a vertex with D <= 2 NT out-neighbours as runs of
// the walk, in k order: thread t takes k = t, then k = NT + t; each v_k goes
// into the position map.  Returns the number of runs (block-uniform).
template <int NT, int MB>
__device__ __forceinline__ i32 hub_runs(int D, i64 bu, i64 gb, const i32* __restrict__ ridx, const i64* __restrict__ G,
                                        const VRec* __restrict__ vrec, BucketMap<MB>& pm, i64* rbase, i32* rstart,
                                        i32* rk, i32* wsum, i32* stot) {
    i32 runs = 0;
    for (int k0 = 0; k0 < D; k0 += NT) {  // uniform over the block
        const int k = k0 + (int)threadIdx.x;
        i32 len = 0, pre = 0;
        i64 bv = 0;
        if (k < D) {
            const i32 v = ridx[bu + k];
            bmap_insert(pm, v, k);
            pre = (i32)(G[bu + k] - gb);
            len = (i32)(G[bu + k + 1] - G[bu + k]);
            { const VRec rv = vrec[v]; bv = rv.off + rv.lo; }
        }
        const i32 cidx = runs + block_scan<NT>(len > 0 ? 1 : 0, wsum, stot);
        if (k < D && len > 0) {
            rbase[cidx] = bv - pre;
            rstart[cidx] = pre;
            if (rk) rk[cidx] = k;
        }
        runs += *stot;
        __syncthreads();  // wsum and the total are reused by the next round
    }
    return runs;
}

__global__ void __launch_bounds__(HT) k_tri1_hub(const i64* __restrict__ roff, const VRec* __restrict__ vrec,
                                                 const i32* __restrict__ ridx, const i32* __restrict__ lo,
                                                 const i64* __restrict__ G, const i32* __restrict__ list, const u32* __restrict__ countp,
                                                 i32 hub_max, i32* __restrict__ C3, u64* __restrict__ bstore,
                                                 const i64* __restrict__ boff, const u32* __restrict__ storep, int defer) {
    const int store = (int)*storep;  // the bitmaps are stored (decided on the device)
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int DM = TRI_HUB_MAX;
    constexpr int NWV = HT / WAVE;
    __shared__ i64 rbase[DM + 1];
    __shared__ i32 rstart[DM + 1];
    __shared__ i32 rk[DM + 1];
    __shared__ BucketMap<10> pm;  // positions of N+(u): 1024 buckets of 4
    __shared__ i32 flags[NWV][WAVE];
    __shared__ i32 Cnt[DM];
    __shared__ i32 wsum[NWV];
    __shared__ i32 stot, sR;
    __shared__ u32 sqe[NWV][HUB_QCAP];
    __shared__ u32 sqkl[NWV][HUB_QCAP];
    __shared__ u64 Bl[HUB_BWORDS];  // rows 0 .. RL-1 of B
    const int wv = threadIdx.x / WAVE;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        if (D > hub_max) continue;  // the global-bitmap kernel takes it (uniform over the block)
        const int W = (D + 63) >> 6;
        const int RL = std::min(D, HUB_BWORDS / W);  // rows of B kept in LDS
        const i64 gb = G[bu];
        const i32 T = (i32)(G[bu + D] - gb);
        u64* const Bg = store ? bstore + boff[u] : nullptr;
        bmap_clear(pm, threadIdx.x, HT);
        for (int q = threadIdx.x; q < RL * W; q += HT) Bl[q] = 0;
        if (Bg)
            for (int q = RL * W + threadIdx.x; q < D * W; q += HT) Bg[q] = 0;
        for (int k = threadIdx.x; k < DM; k += HT) Cnt[k] = 0;
        __threadfence();  // the cleared rows reach L2 before any wavefront's atomics
        __syncthreads();
        // out-neighbour k on thread k mod HT (two rounds when D > HT), runs in k order
        const i32 R = hub_runs<HT>(D, bu, gb, ridx, G, vrec, pm, rbase, rstart, rk, wsum, &stot);
        if (threadIdx.x == 0) {
            sR = R;
            rstart[R] = T;
        }
        __syncthreads();
        const i32 per = ((T + NWV * WAVE - 1) / (NWV * WAVE)) * WAVE;
        HubQueue q{sqe[wv], sqkl[wv], 0};
        run_walk_keyed<4>(std::min(T, wv * per), std::min(T, (wv + 1) * per), rbase, rstart, rk, sR, flags[wv], ridx,
                          [&](bool act, i32, i32 kr, i32 y, i64 e, u64, i32) {
                              const i32 l = act ? bmap_find(pm, y) : -1;
                              const bool hit = l >= 0;
                              if (hit) {
                                  atomicAdd(&Cnt[kr], 1);
                                  atomicAdd(&Cnt[l], 1);
                                  if (kr < RL) atomicOr((unsigned long long*)&Bl[kr * W + (l >> 6)], 1ull << (l & 63));
                              }
                              hub_push(hit, e, ((u32)kr << 16) | (u32)l | (kr < RL ? 0u : HUB_GLOBAL_ROW), q, C3,
                                       Bg, W, defer);
                          });
        hub_flush(q, C3, Bg, W);
        __syncthreads();
        for (int k = threadIdx.x; k < D; k += HT) {
            const i32 c = Cnt[k];
            if (c) atomicAdd(&C3[bu + k], c);
        }
        if (Bg)
            for (int q = threadIdx.x; q < RL * W; q += HT) Bg[q] = Bl[q];
        __threadfence();
        __syncthreads();
    }
}

// ------------------------------------------------------------------ clique / diamond pass

// C3(v, y) - 1 for y in N+(v): y is searched in N+(v) = ridx[from, end),
// starting at `from`, which then moves past it (callers visit y in
// increasing order).  A miss contributes nothing.
__device__ __forceinline__ i64 c3_minus_1(const i32* __restrict__ ridx, const i32* __restrict__ C3, i64& from,
                                          i64 end, i32 y) {
    // galloping from `from`: probes at from, from+1, from+3, ... until past y,
    // then a binary search in the last gap (successive targets are close)
    i64 lo_ = from, step = 1;
    while (lo_ + step - 1 < end && ridx[lo_ + step - 1] < y) {
        lo_ += step;
        step <<= 1;
    }
    const i64 q = lower_bound_dev(ridx, lo_, std::min(lo_ + step - 1, end), y);
    if (q >= end || ridx[q] != y) return 0;
    from = q + 1;
    return (i64)C3[q] - 1;
}

static constexpr int T2_TASK = 8;  // vertices a wavefront takes at a time

__global__ void __launch_bounds__(WT) k_tri2s_wave(const VRec* __restrict__ vrec, const i32* __restrict__ ridx,
                                                   const i64* __restrict__ mir, const i32* __restrict__ list,
                                                   const u32* __restrict__ countp, const i32* __restrict__ C3, i64* __restrict__ k4v,
                                                   i64* __restrict__ d13, i64* __restrict__ ek,
                                                   const u64* __restrict__ bstore, const i64* __restrict__ boff,
    const u32* __restrict__ storep) {
    if (!*storep) return;  // the bitmaps were not stored: the fallback kernels count
    const u32 count = *countp;  // the tier size, written on the device
    // Each wavefront works alone, on T2_TASK consecutive vertices at a time,
    // packed into rounds: consecutive vertices whose out-degrees sum to at
    // most 64 share the 64 lanes, vertex g's rows k on lanes off_g + k, its
    // bitmap rows shifted to those lanes' bit positions (the 64 x 64
    // transpose then transposes every vertex's block on its own).  Edge by
    // edge over the induced subgraph H on N+(u): lane k takes the edges
    // (k, l), l in B_k (l > k).  With A = B | B^T, edge (k, l) lies on
    // c = |A_k & A_l| triangles of H; k keeps its sums in registers, l's
    // arrive by LDS atomics.  The triangles of H through k are half its sum
    // of c, and u's 4-cliques the sum over its edges divided by three.
    // Diamonds: v_k gets C3(u, v_l) - 1 per edge at k; u gets C3(v_k, v_l) - 1
    // per edge, found by a galloping search of v_l in N+(v_k).
    constexpr int NW = WT / WAVE;
    __shared__ u64 sA[NW][WAVE];
    __shared__ i32 sL[NW][WAVE];
    __shared__ i32 sc3[NW][WAVE];
    __shared__ u32 st2[NW][WAVE];
    __shared__ u32 sdv[NW][WAVE];
    __shared__ i32 sflag[NW][WAVE];
    const int wid = threadIdx.x / WAVE;
    const int lane = lane_id();
    const u64 le = lane == WAVE - 1 ? ~0ull : ((1ull << (lane + 1)) - 1);
    // tasks from the end of the list first: the list follows rank, and the
    // vertices of high out-degree (long tasks) come last in it
    const i64 ntasks = ((i64)count + T2_TASK - 1) / T2_TASK;
    for (i64 tj = (i64)blockIdx.x * NW + wid; tj < ntasks; tj += (i64)gridDim.x * NW) {
        const i64 t0 = (ntasks - 1 - tj) * T2_TASK;
        const int ntask = (int)std::min<i64>(T2_TASK, (i64)count - t0);
        // lanes i < ntask: vertex t0 + i
        i64 u_i = 0, bu_i = 0, bo_i = 0;
        i32 D_i = 0;
        if (lane < ntask) {
            u_i = list[t0 + lane];
            const VRec r = vrec[u_i];
            bu_i = r.off + r.lo;
            D_i = r.deg - r.lo;
            bo_i = boff[u_i];
        }
        for (int next = 0; next < ntask;) {
            // this round: vertices next .. next + P - 1, the longest run whose
            // out-degrees sum to at most 64 (every out-degree is at most 64)
            const i32 dd = (lane >= next && lane < ntask) ? D_i : 0;
            const i32 incl = wave_incl_scan_i32(dd);
            const u64 inr = __ballot(lane >= next && lane < ntask && incl <= WAVE);
            const int P = __popcll(inr);
            const i32 excl = incl - dd;
            // lane L belongs to the vertex g whose lanes [excl_g, excl_g + D_g) hold it
            lds_put(&sflag[wid][lane], 0);
            wave_lds_fence();
            if ((inr >> lane) & 1ull) lds_put(&sflag[wid][excl], 1);
            wave_lds_fence();
            const u64 starts = __ballot(lds_get(&sflag[wid][lane]) != 0);
            const i32 used = __builtin_amdgcn_readlane(incl, next + P - 1);
            const int g = next + __popcll(starts & le) - 1;  // vertex of this lane (valid when lane < used)
            const bool act = lane < used;
            const i64 u = __shfl(u_i, g, WAVE);
            const i64 bu = __shfl(bu_i, g, WAVE);
            const i64 bo = __shfl(bo_i, g, WAVE);
            const i32 off_g = __shfl(excl, g, WAVE);
            const i32 k = lane - off_g;
            u64 Bk = 0;
            i32 vk = 0, c3k = 0;
            i64 mk = 0;
            if (act) {
                Bk = bstore[bo + k] << off_g;
                vk = ridx[bu + k];
                c3k = C3[bu + k];
                mk = mir[bu + k];  // the entry (v_k, u)
            }
            const u64 Ak = Bk | wave_transpose64(Bk);
            sA[wid][lane] = Ak;
            lds_put(&sL[wid][lane], vk);
            lds_put(&sc3[wid][lane], c3k);
            lds_put(reinterpret_cast<i32*>(&st2[wid][lane]), 0);
            lds_put(reinterpret_cast<i32*>(&sdv[wid][lane]), 0);
            wave_lds_fence();
            u32 tk = 0, dk = 0;
            i64 R = 0, du = 0;
            if (act) {
                const VRec rec = vrec[vk];
                i64 from = rec.off + rec.lo;
                const i64 end = rec.off + rec.deg;
                const u32 ck = (u32)(c3k - 1);
                FOR_BITS(Bk, l, {
                    const u32 c = (u32)__popcll(Ak & sA[wid][l]);
                    tk += c;
                    R += c;
                    dk += (u32)(lds_get(&sc3[wid][l]) - 1);
                    if (c) atomicAdd(&st2[wid][l], c);
                    if (ck) atomicAdd(&sdv[wid][l], ck);
                    du += c3_minus_1(ridx, C3, from, end, lds_get(&sL[wid][l]));
                });
            }
            wave_lds_fence();
            if (act) {
                const i64 kv = (i64)((tk + st2[wid][lane]) >> 1);
                const i64 dv = (i64)dk + sdv[wid][lane];
                if (kv | dv) ek[mk] = (dv << EK_SHIFT) | kv;
            }
            // per-vertex totals: runs of equal g among the active lanes
            const WaveRuns wr = wave_runs(g, act);
            R = run_total(R, wr);
            du = run_total(du, wr);
            if (wr.tail) {
                if (R) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)(R / 3));
                if (du) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)du);
            }
            wave_lds_fence();  // the next round overwrites the rows
            next += P;
        }
    }
}

// LDS tier: edge-parallel over the induced subgraph H on N+(u).  With A =
// B | B^T (full adjacency rows of H), an edge (k, l) of H lies on
// c = |A_k & A_l| triangles of H, each a 4-clique with u; the triangles of H
// through k are half the sum of c over its edges, and its 4-clique count of u
// is the sum over edges divided by three.  Threads take the 64-bit words of
// B (each at most 64 edges), so the work does not pile up on the rows of
// popular vertices; per-vertex sums gather in LDS.  The diamond term of u
// comes from k_tri2_du_lds (a search per edge here costs more than walking
// the out-lists again).
__global__ void __launch_bounds__(LT) k_tri2s_lds(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                  const i32* __restrict__ lo, const i64* __restrict__ mir,
                                                  const i32* __restrict__ list, const u32* __restrict__ countp,
                                                  const i32* __restrict__ C3, i64* __restrict__ k4v,
                                                  i64* __restrict__ ek,
                                                  const u64* __restrict__ bstore, const i64* __restrict__ boff,
    const u32* __restrict__ storep) {
    if (!*storep) return;  // the bitmaps were not stored: the fallback kernels count
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int DM = TRI_LDS_MAX;
    constexpr int WM = DM / 64;
    __shared__ u64 B[DM * WM];
    __shared__ u64 A[DM * WM];
    __shared__ i32 L[DM];
    __shared__ i32 c3u[DM];
    __shared__ u32 t2[DM];   // twice the triangles of H through k: below 2 * 511 * 510
    __shared__ u32 dvs[DM];  // diamonds of v_k: below 511 * 2^21
    __shared__ i64 red[1];
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        const int W = (D + 63) >> 6;
        const u64* src = bstore + boff[u];
        for (int q = threadIdx.x; q < D * W; q += LT) B[q] = src[q];
        if (threadIdx.x < D) {
            L[threadIdx.x] = ridx[bu + threadIdx.x];
            c3u[threadIdx.x] = C3[bu + threadIdx.x];
            t2[threadIdx.x] = 0;
            dvs[threadIdx.x] = 0;
        }
        if (threadIdx.x == 0) red[0] = 0;
        __syncthreads();
        // A = B | B^T, 64 x 64 blocks: wavefront wv takes the blocks (bi, bj)
        // with bi * W + bj = wv (mod LT / 64); lane = row in the block
        for (int blk = threadIdx.x / WAVE; blk < W * W; blk += LT / WAVE) {
            const int bi = blk / W, bj = blk % W;
            const int row = bi * 64 + lane_id();
            const u64 m = row < D ? B[row * W + bj] : 0ull;
            const u64 t = wave_transpose64(m);  // column bj * 64 + lane of the block
            const int col = bj * 64 + lane_id();
            if (col < D) A[col * W + bi] = t | B[col * W + bi];
        }
        __syncthreads();
        i64 R = 0;
        for (int i = threadIdx.x; i < D * W; i += LT) {
            const int k = i / W, wa = i - k * W;
            u64 bits = B[i];
            if (!bits) continue;
            u64 Ak[WM];
#pragma unroll
            for (int z = 0; z < WM; ++z) Ak[z] = z < W ? A[k * W + z] : 0ull;
            const u32 ck = (u32)(c3u[k] - 1);
            u32 tk = 0, dk = 0;
            FOR_BITS(bits, bb, {
                const int l = wa * 64 + bb;
                const u64* Al = A + l * W;
                u32 c = 0;
                for (int z = 0; z < W; ++z) c += (u32)__popcll(Ak[z] & Al[z]);
                tk += c;
                dk += (u32)(c3u[l] - 1);
                if (c) atomicAdd(&t2[l], c);
                if (ck) atomicAdd(&dvs[l], ck);
                R += c;
            });
            if (tk) atomicAdd(&t2[k], tk);
            if (dk) atomicAdd(&dvs[k], dk);
        }
        R = wave_sum(R);
        if (lane_id() == 0 && R) atomicAdd((unsigned long long*)&red[0], (unsigned long long)R);
        __syncthreads();
        const int k = threadIdx.x;
        if (k < D) {
            const i64 kv = t2[k] >> 1, dv = dvs[k];
            if (kv | dv) ek[mir[bu + k]] = (dv << EK_SHIFT) | kv;
        }
        if (threadIdx.x == 0 && red[0]) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)(red[0] / 3));
        __syncthreads();
    }
}

// |Ak & Al| over the first W words of two rows, unrolled with constant
// indices so that Ak stays in registers (a loop bounded by W alone indexes Ak
// at run time and moves it to scratch memory).
template <int WM>
__device__ __forceinline__ u32 popc_and_row(const u64 (&Ak)[WM], const u64* Al, int W) {
    u32 c = 0;
#pragma unroll
    for (int z = 0; z < WM; ++z)
        if (z < W) c += (u32)__popcll(Ak[z] & Al[z]);
    return c;
}

// Hub tier of the clique pass (D <= hub_max <= TRI_HUB_MAX): as the LDS tier,
// with A = B | B^T (up to 1024 x 16 words) in LDS and B itself read from the
// workspace rows the hub triangle pass wrote (each word once, when its edges
// are taken, and once for the transpose).
__global__ void __launch_bounds__(HT) k_tri2s_hub(const i64* __restrict__ roff, const i32* __restrict__ lo,
                                                  const i64* __restrict__ mir, const i32* __restrict__ list,
                                                  const u32* __restrict__ countp, i32 hub_max, const i32* __restrict__ C3,
                                                  i64* __restrict__ k4v, i64* __restrict__ ek,
                                                  const u64* __restrict__ bstore, const i64* __restrict__ boff,
    const u32* __restrict__ storep) {
    if (!*storep) return;  // the bitmaps were not stored: the fallback kernels count
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int DM = TRI_HUB_MAX;
    constexpr int WM = DM / 64;
    __shared__ u64 A[DM * WM];
    __shared__ i32 c3u[DM];
    __shared__ u32 t2[DM];   // twice the triangles of H through k: below 2 * 1087 * 1086
    __shared__ u32 dvs[DM];  // diamonds of v_k: below 1087 * 2^21
    __shared__ i64 red[1];
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        if (D > hub_max) continue;  // uniform over the block
        const int W = (D + 63) >> 6;
        const u64* const B = bstore + boff[u];
        for (int k = threadIdx.x; k < D; k += HT) {
            c3u[k] = C3[bu + k];
            t2[k] = 0;
            dvs[k] = 0;
        }
        if (threadIdx.x == 0) red[0] = 0;
        // A = B | B^T, 64 x 64 blocks: wavefront wv takes the blocks (bi, bj)
        // with bi * W + bj = wv (mod HT / 64); lane = row in the block
        for (int blk = threadIdx.x / WAVE; blk < W * W; blk += HT / WAVE) {
            const int bi = blk / W, bj = blk % W;
            const int row = bi * 64 + lane_id();
            const u64 m = row < D ? B[(i64)row * W + bj] : 0ull;
            const u64 t = wave_transpose64(m);  // column bj * 64 + lane of the block
            const int col = bj * 64 + lane_id();
            if (col < D) A[col * W + bi] = t | B[(i64)col * W + bi];
        }
        __syncthreads();
        i64 R = 0;
        for (int i = threadIdx.x; i < D * W; i += HT) {
            const int k = i / W, wa = i - k * W;
            u64 bits = B[i];
            if (!bits) continue;
            u64 Ak[WM];
#pragma unroll
            for (int z = 0; z < WM; ++z) Ak[z] = z < W ? A[k * W + z] : 0ull;
            const u32 ck = (u32)(c3u[k] - 1);
            u32 tk = 0, dk = 0;
            FOR_BITS(bits, bb, {
                const int l = wa * 64 + bb;
                const u64* Al = A + l * W;
                const u32 c = popc_and_row<WM>(Ak, Al, W);
                tk += c;
                dk += (u32)(c3u[l] - 1);
                if (c) atomicAdd(&t2[l], c);
                if (ck) atomicAdd(&dvs[l], ck);
                R += c;
            });
            if (tk) atomicAdd(&t2[k], tk);
            if (dk) atomicAdd(&dvs[k], dk);
        }
        R = wave_sum(R);
        if (lane_id() == 0 && R) atomicAdd((unsigned long long*)&red[0], (unsigned long long)R);
        __syncthreads();
        for (int k = threadIdx.x; k < D; k += HT) {
            const i64 kv = t2[k] >> 1, dv = dvs[k];
            if (kv | dv) ek[mir[bu + k]] = (dv << EK_SHIFT) | kv;
        }
        if (threadIdx.x == 0 && red[0]) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)(red[0] / 3));
        __syncthreads();
    }
}

// Diamond term of u for the LDS tier: over the triangles (u, v_k, v_l), the
// number of other triangles on the opposite edge, C3(v_k, v_l) - 1.  The
// out-lists N+(v_k) are walked again as in the triangle pass; a hit y = v_l
// sits at the walked entry e, whose C3 is final now.
// NT threads take one vertex with D <= DM <= 2 NT; MB: the position map's
// bucket bits.  The hub instance skips the vertices above hub_max.
template <int NT, int DM, int MB>
__global__ void __launch_bounds__(NT) k_tri2_du_lds(const i64* __restrict__ roff, const VRec* __restrict__ vrec, const i32* __restrict__ ridx,
                                                    const i32* __restrict__ lo, const i64* __restrict__ G,
                                                    const i32* __restrict__ list, const u32* __restrict__ countp, i32 hub_max,
                                                    const i32* __restrict__ C3, i64* __restrict__ d13,
    const u32* __restrict__ storep) {
    if (!*storep) return;  // the bitmaps were not stored: the fallback kernels count
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int NWV = NT / WAVE;
    __shared__ i64 rbase[DM + 1];
    __shared__ i32 rstart[DM + 1];
    __shared__ BucketMap<MB> pm;
    __shared__ i32 flags[NWV][WAVE];
    __shared__ i32 wsum[NWV];
    __shared__ i32 stot, sR;
    __shared__ i64 part[NWV];
    const int wv = threadIdx.x / WAVE;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        if (D > hub_max) continue;  // uniform over the block
        const i64 gb = G[bu];
        const i32 T = (i32)(G[bu + D] - gb);
        bmap_clear(pm, threadIdx.x, NT);
        __syncthreads();
        const i32 R = hub_runs<NT>(D, bu, gb, ridx, G, vrec, pm, rbase, rstart, (i32*)nullptr, wsum, &stot);
        if (threadIdx.x == 0) {
            sR = R;
            rstart[R] = T;
        }
        __syncthreads();
        const i32 per = ((T + NWV * WAVE - 1) / (NWV * WAVE)) * WAVE;
        i64 du = 0;
        run_walk<4>(std::min(T, wv * per), std::min(T, (wv + 1) * per), rbase, rstart, sR, flags[wv], ridx,
                    [&](bool act, i32, i32, i32 y, i64 e, u64, i32) {
                        if (act && bmap_find(pm, y) >= 0) du += (i64)C3[e] - 1;
                    });
        du = block_sum<NT>(du, part);
        if (threadIdx.x == 0 && du) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)du);
    }
}

// Bitmap words of every vertex of the wave and LDS tiers (D x ceil(D/64)).
__global__ void k_bitmap_words(const i64* __restrict__ roff, const i32* __restrict__ lo, i64 n, i64 lds_max,
                               i64* __restrict__ words,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (i64)gridDim.x * blockDim.x) {
        const i64 D = roff[u + 1] - roff[u] - lo[u];
        words[u] = (D >= 2 && D <= lds_max) ? D * ((D + 63) / 64) : 0;
    }
}

// ------------------------------------------------------------------ launchers

static inline unsigned tgrid(i64 work, i64 per_block) {
    return (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(std::max<i64>(work, 1), per_block), 65536));
}

hipError_t launch_bitmap_offsets(i64 n, RawWs& w, i64 lds_max, hipStream_t s) {
    hipLaunchKernelGGL(k_bitmap_words, dim3(tgrid(n, 256)), dim3(256), 0, s, w.roff, w.lo, n, lds_max, w.bcnt,
                       (const u32*)&w.plan->err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_exclusive_i64(w.bcnt, w.boff, n, w.partials, s);
}

// Grids of the tier launches, from bounds on the tier sizes (the sizes
// themselves are on the device): a vertex of out-degree above D has more
// than D of the nnz / 2 oriented edges.
static inline unsigned tier_grid(i64 n, i64 nnz, int tier, i64 per_block, i64 cap) {
    const i64 bound = tier == 0 ? n : std::min<i64>(n, nnz / (tier == 1 ? 2 * TRI_WAVE_MAX : 2 * TRI_LDS_MAX) + 1);
    return (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(std::max<i64>(bound, 1), per_block), cap));
}

hipError_t launch_tri1_stored(i64 n, i64 nnz, RawWs& w, hipStream_t s, int tier, i64 hub_max) {
    const u32* const cnt = w.plan->n_tri;
    const u32* const stp = &w.plan->stored;
    const int defer = nnz <= (i64)0xffffffffLL;  // entry indices fit the 32-bit queue
    if (tier == 0) {
        if (n <= ((i64)1 << 28))  // position-map keys (v, slot) fit 31 bits
            hipLaunchKernelGGL(k_tri1_wave<true>, dim3(tier_grid(n, nnz, 0, WT / WAVE * 8, 65536)), dim3(WT), 0, s,
                               w.vrec, w.ridx, w.tri_list, cnt + 0, w.C3, w.bstore, w.boff, stp, defer);
        else
            hipLaunchKernelGGL(k_tri1_wave<false>, dim3(tier_grid(n, nnz, 0, WT / WAVE, 65536)), dim3(WT), 0, s,
                               w.vrec, w.ridx, w.tri_list, cnt + 0, w.C3, w.bstore, w.boff, stp, defer);
    }
    if (tier == 1)
        hipLaunchKernelGGL(k_tri1_lds, dim3(tier_grid(n, nnz, 1, 1, 65536)), dim3(LT), 0, s, w.roff, w.vrec, w.ridx,
                           w.lo, w.G, w.tri_list + n, cnt + 1, w.C3, w.bstore, w.boff, stp, defer);
    if (tier == 2 && hub_max > 0)  // the hub tier's vertices of the last tier list
        hipLaunchKernelGGL(k_tri1_hub, dim3(tier_grid(n, nnz, 2, 1, 4096)), dim3(HT), 0, s, w.roff, w.vrec, w.ridx,
                           w.lo, w.G, w.tri_list + 2 * n, cnt + 2, (i32)hub_max, w.C3, w.bstore, w.boff, stp, defer);
    return hipGetLastError();
}

hipError_t launch_tri2_stored(i64 n, i64 nnz, RawWs& w, hipStream_t s, int tier, i64 hub_max) {
    const u32* const cnt = w.plan->n_tri;
    const u32* const stp = &w.plan->stored;
    if (tier == 0)
        hipLaunchKernelGGL(k_tri2s_wave, dim3(tier_grid(n, nnz, 0, WT / WAVE * T2_TASK, 65536)), dim3(WT), 0, s,
                           w.vrec, w.ridx, w.mir, w.tri_list, cnt + 0, w.C3, w.k4v, w.d13, w.ek, w.bstore, w.boff, stp);
    if (tier == 1) {
        hipLaunchKernelGGL(k_tri2s_lds, dim3(tier_grid(n, nnz, 1, 1, 65536)), dim3(LT), 0, s, w.roff, w.ridx, w.lo,
                           w.mir, w.tri_list + n, cnt + 1, w.C3, w.k4v, w.ek, w.bstore, w.boff, stp);
        hipLaunchKernelGGL((k_tri2_du_lds<LT, TRI_LDS_MAX, 9>), dim3(tier_grid(n, nnz, 1, 1, 65536)), dim3(LT), 0, s, w.roff,
                           w.vrec, w.ridx, w.lo, w.G, w.tri_list + n, cnt + 1, (i32)TRI_LDS_MAX, w.C3, w.d13, stp);
    }
    if (tier == 2 && hub_max > 0) {
        hipLaunchKernelGGL(k_tri2s_hub, dim3(tier_grid(n, nnz, 2, 1, 4096)), dim3(HT), 0, s, w.roff, w.lo, w.mir,
                           w.tri_list + 2 * n, cnt + 2, (i32)hub_max, w.C3, w.k4v, w.ek, w.bstore, w.boff, stp);
        hipLaunchKernelGGL((k_tri2_du_lds<HT, TRI_HUB_MAX, 10>), dim3(tier_grid(n, nnz, 2, 1, 4096)), dim3(HT), 0, s, w.roff,
                           w.vrec, w.ridx, w.lo, w.G, w.tri_list + 2 * n, cnt + 2, (i32)hub_max, w.C3, w.d13, stp);
    }
    return hipGetLastError();
}

}  // namespace fglt
