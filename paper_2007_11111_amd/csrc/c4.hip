// c4.hip -- the 4-cycle pass: per-vertex 4-cycle counts (C4,2 e / 2, Lemma 5)
// with their attribution to every vertex of the cycle.
//
// Every 4-cycle is found once, from its highest-ranked vertex u, as a pair of
// rank-ordered wedges u - v - w and u - v' - w with v, v', w < u.  With c(w)
// the number of wedges of u that end in w (the common neighbours of u and w
// that rank below u), u gains sum_w C(c(w), 2), each end w gains C(c(w), 2),
// and each middle v gains, over its wedges u - v - w, the sum of c(w) - 1.
//
// Tiers by the wedge count W(u) = sum over v in N-(u) of |N(v) below u|:
//   wave    W <= 128     one wavefront per vertex, 256-slot LDS hash
//   block   W <= 2048    one 256-thread workgroup per vertex, 4096-slot hash
//   hash    W <= 16384   one 1024-thread workgroup per vertex, 32768-slot hash
//                        of packed (end rank, count) words
//   window  beyond       dense LDS counters over windows of consecutive ranks;
//                        one workgroup per vertex (all windows in turn) when
//                        its middles fit one 1024-thread chunk, else one per
//                        (vertex, window)
// The two large-workgroup tiers flatten the wedge runs of up to 1024 middles
// (middle v of u contributes the run of N(v) below u, or its part inside the
// window) with one block scan and walk them 64 consecutive items per
// wavefront step, so the reads of each run are coalesced.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "walk.h"

namespace fglt {

static constexpr int PT = 256;

// ------------------------------------------------------------ small tiers

// Wedge items of vertex u (N- entries in [b, m)), visited in increasing
// order g: the entry q = (u, v) holding item g is found by one binary search
// over the work prefix G for the first item, then by moving forward; the
// wedge end is w = the (g - G[q])-th neighbour of v.  Row v starts at
// mir[q] - rpos[q] (the mirror (v, u) sits rpos[q] = G[q+1] - G[q] entries
// into it), so no lookup of v's row is needed.
struct WedgeCursor {
    i64 q = -1, qs = 0, qe = 0, rs = 0;  // entry, its items [qs, qe), row start of its middle
    // item g alone: one binary search (no cursor state kept)
    __device__ __forceinline__ i32 once(const i64* __restrict__ G, const i64* __restrict__ mir,
                                        const i32* __restrict__ ridx, i64 b, i64 m, i64 g) {
        q = last_le_dev(G, b, m - 1, g);
        return ridx[mir[q] - G[q + 1] + g];
    }
    __device__ __forceinline__ i32 at(const i64* __restrict__ G, const i64* __restrict__ mir,
                                      const i32* __restrict__ ridx, i64 b, i64 m, i64 g) {
        if (q < 0 || g >= qe) {
            q = q < 0 ? last_le_dev(G, b, m - 1, g) : q + 1;
            while (G[q + 1] <= g) ++q;  // skip middles without wedges
            qs = G[q];
            qe = G[q + 1];
            rs = mir[q] - (qe - qs);
        }
        return ridx[rs + (g - qs)];
    }
};

// LDS-hash tiers.  WAVES_PER_U = 1: one wavefront per vertex (4 per block,
// 256-slot table each); WAVES_PER_U = 4: the whole block on one vertex with a
// 4096-slot table.
template <int WAVES_PER_U, int HSLOTS>
__global__ void __launch_bounds__(PT) k_c4_hash(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                const i32* __restrict__ lo, const i64* __restrict__ G,
                                                const i64* __restrict__ mir,
                                                const i32* __restrict__ list, const u32* __restrict__ countp, i64* __restrict__ c4v) {
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int NW = PT / WAVE;
    constexpr int GROUPS = NW / WAVES_PER_U;  // vertices per block
    constexpr int GT = WAVES_PER_U * WAVE;    // threads per vertex
    constexpr int LMAX = HSLOTS / 2;  // middles of a vertex: at most its wedge count
    __shared__ i32 hk[GROUPS][HSLOTS];
    __shared__ i32 hc[GROUPS][HSLOTS];
    __shared__ i32 msum[GROUPS][LMAX];  // per-middle sums of pass C (at most W^2 < 2^31)
    __shared__ i64 red[GROUPS];
    const int grp = threadIdx.x / GT;
    const int gt = threadIdx.x % GT;
    const u32 mask = HSLOTS - 1;
    // a one-wavefront group shares no LDS with the other groups: it runs its
    // own vertices with wavefront fences; a whole-block group synchronizes
    auto group_sync = [&]() {
        if (WAVES_PER_U == 1) wave_lds_fence();
        else __syncthreads();
    };
    for (i64 it = (i64)blockIdx.x * GROUPS + grp; it < (i64)count; it += (i64)gridDim.x * GROUPS) {
        const i64 u = list[it];
        const i64 b = roff[u];
        const i64 m = b + lo[u];
        const i64 gb = G[b];
        const i64 W = G[m] - gb;
        for (int s = gt; s < HSLOTS; s += GT) {
            hk[grp][s] = -1;
            hc[grp][s] = 0;
        }
        for (int s = gt; s < LMAX; s += GT) msum[grp][s] = 0;
        if (gt == 0) red[grp] = 0;
        group_sync();
        // a workgroup's threads take ipt consecutive items each (one search,
        // then a forward walk); a wavefront's lanes (at most two items each)
        // take every GT-th item with a search per item
        const i64 ipt = (W + GT - 1) / GT;
        const i64 t0 = WAVES_PER_U == 1 ? gt : gt * ipt;
        const i64 ts = WAVES_PER_U == 1 ? GT : 1;
        // pass A: count wedge ends
        {
            WedgeCursor cur;
            for (i64 s = 0; s < ipt; ++s) {
                const i64 t = t0 + s * ts;
                if (t >= W) break;
                const i32 w = WAVES_PER_U == 1 ? cur.once(G, mir, ridx, b, m, gb + t)
                                               : cur.at(G, mir, ridx, b, m, gb + t);
                hash_add(hk[grp], hc[grp], mask, w);
            }
        }
        group_sync();
        // pass C: cnt(w) - 1 to the middle vertex of every wedge; the sums go
        // to LDS per middle when the vertex's middles fit the array (a vertex
        // may have many middles without wedges), else straight to memory
        const bool lsum = m - b <= LMAX;
        WedgeCursor cur;
        for (i64 s = 0; s < ipt; ++s) {  // items t0 + s * ts rise with the lane, so do their entries
            const i64 t = t0 + s * ts;
            const bool act = t < W;
            i64 q = -1, val = 0;
            if (act) {
                const i32 w = WAVES_PER_U == 1 ? cur.once(G, mir, ridx, b, m, gb + t)
                                               : cur.at(G, mir, ridx, b, m, gb + t);
                q = cur.q;
                val = hash_get(hk[grp], hc[grp], mask, w) - 1;
            }
            val = wave_seg_scan(val, q);
            if (wave_seg_tail(q, act) && val) {
                if (lsum) atomicAdd(&msum[grp][q - b], (i32)val);
                else atomicAdd((unsigned long long*)&c4v[ridx[q]], (unsigned long long)val);
            }
        }
        // pass B: C(cnt, 2) to u and to w (after the gathers, so that these
        // atomics hold back no load of pass C)
        i64 accu = 0;
        for (int s = gt; s < HSLOTS; s += GT) {
            const i32 w = hk[grp][s];
            if (w >= 0) {
                const i64 c = hc[grp][s];
                if (c >= 2) {
                    const i64 pr = c * (c - 1) / 2;
                    accu += pr;
                    atomicAdd((unsigned long long*)&c4v[w], (unsigned long long)pr);
                }
            }
        }
        accu = wave_sum(accu);
        if (lane_id() == 0 && accu) atomicAdd((unsigned long long*)&red[grp], (unsigned long long)accu);
        group_sync();
        // the middles' sums, one global atomic per middle
        if (lsum) {
            for (i64 k = gt; k < m - b; k += GT) {
                const i32 v = msum[grp][k];
                if (v) atomicAdd((unsigned long long*)&c4v[ridx[b + k]], (unsigned long long)v);
            }
        }
        if (gt == 0 && red[grp]) atomicAdd((unsigned long long*)&c4v[u], (unsigned long long)red[grp]);
        group_sync();
    }
}

// ------------------------------------------------------------ large-workgroup tiers

static constexpr int CB_THREADS = 1024;
static constexpr int CB_NWV = CB_THREADS / WAVE;

__device__ __forceinline__ i32 wave_min_i32(i32 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ __forceinline__ i32 wave_max_i32(i32 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return v;
}

// LDS state of the flattened wedge runs of one chunk of middles.
struct RunLds {
    i64 rbase[CB_THREADS + 1];  // item t of run r sits at ridx[rbase[r] + t]
    i32 rk[CB_THREADS + 1];     // middle of run r, as its index within the chunk
    i32 rstart[CB_THREADS + 1]; // first item of run r; rstart[nruns] = item count
    i32 flags[CB_NWV][WAVE];    // run-start exchange rows of the walk
    i64 wsum[CB_NWV];
    i64 total;
    i32 nruns;
};

// Compacts the wedge runs of middles c0 .. c0+1023 of the current vertex
// (middle k < L).  run(k, s0, len) gives middle k's wedge ends
// ridx[s0 .. s0+len).  The non-empty runs are kept in middle order; one
// block scan of (items << 16 | non-empty) gives both prefixes.  Returns the
// item count.  Every thread of the block calls it.
template <class RunOf>
__device__ __forceinline__ i32 flatten_runs(i32 L, i32 c0, RunOf&& run, RunLds& R) {
    const i32 k = c0 + (i32)threadIdx.x;
    i32 len = 0;
    i64 s0 = 0;
    if (k < L) run(k, s0, len);
    const i64 packed = ((i64)len << 16) | (len > 0 ? 1 : 0);
    const i64 pre = block_scan<CB_THREADS>(packed, R.wsum, &R.total);
    const i64 tot = R.total;
    const i32 items_before = (i32)(pre >> 16), runs_before = (i32)(pre & 0xffff);
    if (len > 0) {
        R.rbase[runs_before] = s0 - items_before;
        R.rk[runs_before] = (i32)threadIdx.x;
        R.rstart[runs_before] = items_before;
    }
    const i32 T = (i32)(tot >> 16);
    if (threadIdx.x == 0) {
        R.nruns = (i32)(tot & 0xffff);
        R.rstart[tot & 0xffff] = T;
    }
    __syncthreads();
    return T;
}

// Items of the chunk handled by wavefront wv: [ta, tb), a multiple of 64 wide.
__device__ __forceinline__ void wave_share(i32 T, i32& ta, i32& tb) {
    const i32 per = ((T + CB_THREADS - 1) / CB_THREADS) * WAVE;
    const i32 wv = (i32)threadIdx.x / WAVE;
    ta = min(T, wv * per);
    tb = min(T, (wv + 1) * per);
}

// Pass C walk: every wedge item gives cnt(w) - 1 to its middle.  The sum of
// each run's piece in a wavefront step comes from a wave prefix sum and the
// run-start mask and goes to the middle's LDS sum msum[k]; the caller moves
// the sums to global memory once per chunk (or per vertex), so that no global
// atomic sits between the gathers of the walk.
// SMALL: every count is below 2^16, so a wavefront's prefix sums fit 32 bits
// and the DPP scan applies.
__device__ __forceinline__ void lds_add(i64* p, i64 v) { atomicAdd((unsigned long long*)p, (unsigned long long)v); }
__device__ __forceinline__ void lds_add(u32* p, i64 v) { atomicAdd(p, (u32)v); }  // sums below 2^32

template <bool SMALL, class MS, class Get>
__device__ __forceinline__ void attribute_middles(i32 T, RunLds& R, const i32* __restrict__ ridx, MS* msum,
                                                  Get&& get) {
    i32 ta, tb;
    wave_share(T, ta, tb);
    const int l = lane_id();
    const int wv = (int)threadIdx.x / WAVE;
    run_walk_keyed<4>(ta, tb, R.rbase, R.rstart, R.rk, R.nruns, R.flags[wv], ridx,
                      [&](bool act, i32 t, i32 kr, i32 w, i64, u64 mask, i32 tend) {
                    // a run piece's sum is P(tail) - P(before its head): the tail
                    // adds the inclusive prefix, the head takes away its exclusive one
                    i64 P, val;
                    if (SMALL) {
                        const i32 v = act ? (i32)get(w) - 1 : 0;
                        P = wave_incl_scan_i32(v);
                        val = v;
                    } else {
                        val = act ? (i64)get(w) - 1 : 0;
                        P = val;
#pragma unroll
                        for (int o = 1; o < WAVE; o <<= 1) {
                            const i64 y = __shfl_up(P, o, WAVE);
                            if (l >= o) P += y;
                        }
                    }
                    const bool head = act && (l == 0 || ((mask >> l) & 1ull));
                    const bool tail = act && (l == WAVE - 1 || ((mask >> (l + 1)) & 1ull) || t + 1 >= tend);
                    const i64 add = (tail ? P : 0) - (head ? P - val : 0);
                    if (add) lds_add(&msum[kr], add);
                });
}

// ---- hash tier: packed words (end rank << cb) | count, 0 when empty.  The
// count of an end is at most |N-(u)|, which the tier assignment keeps below
// 2^cb; at most 16384 distinct ends keep the table at most half full.

static constexpr int C4H_BITS = 15;
static constexpr int C4H_SLOTS = 1 << C4H_BITS;  // 128 KiB

__device__ __forceinline__ u32 c4h_slot(i32 w) { return ((u32)w * 2654435761u) >> (32 - C4H_BITS); }

__device__ __forceinline__ void c4h_add(u32* tab, i32 w, int cb) {
    u32 h = c4h_slot(w);
    {  // the first slot in straight-line code; the loop below only on a collision
        u32 e = tab[h];
        if (e == 0) {
            e = atomicCAS(&tab[h], 0u, ((u32)w << cb) | 1u);
            if (e == 0) return;
        }
        if ((e >> cb) == (u32)w) {
            atomicAdd(&tab[h], 1u);
            return;
        }
        h = (h + 1) & (C4H_SLOTS - 1);
    }
    while (true) {
        u32 e = tab[h];
        if (e == 0) {
            const u32 old = atomicCAS(&tab[h], 0u, ((u32)w << cb) | 1u);
            if (old == 0) return;
            e = old;
        }
        if ((e >> cb) == (u32)w) {  // the key bits of a word never change once set
            atomicAdd(&tab[h], 1u);
            return;
        }
        h = (h + 1) & (C4H_SLOTS - 1);
    }
}

__device__ __forceinline__ u32 c4h_get(const u32* tab, i32 w, int cb) {
    u32 h = c4h_slot(w);
    u32 e = tab[h];
    if (e != 0 && (e >> cb) != (u32)w) {
        do {
            h = (h + 1) & (C4H_SLOTS - 1);
            e = tab[h];
        } while (e != 0 && (e >> cb) != (u32)w);
    }
    return e & ((1u << cb) - 1u);  // 0 for an empty slot
}

__global__ void __launch_bounds__(CB_THREADS) k_c4_hashbig(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                           const i32* __restrict__ lo, const i32* __restrict__ rpos,
                                                           const i64* __restrict__ mir,
                                                           const i32* __restrict__ list, const u32* __restrict__ countp,
                                                           u32* __restrict__ job_ctr, int cb, i64* __restrict__ c4v) {
    const u32 count = *countp;  // the tier size, written on the device
    __shared__ u32 tab[C4H_SLOTS];
    __shared__ RunLds R;
    __shared__ i64 msum[CB_THREADS];
    __shared__ i64 sj, red;
    const u32 cmask = (1u << cb) - 1u;
    for (int q = threadIdx.x; q < C4H_SLOTS; q += CB_THREADS) tab[q] = 0;
    msum[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        sj = atomicAdd(job_ctr, 1u);
        red = 0;
    }
    __syncthreads();
    while (true) {
        const i64 j = sj;
        if (j >= (i64)count) break;
        u32 nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(job_ctr, 1u);  // consumed at the end of this job
        const i32 u = list[j];
        const i64 b = roff[u];
        const i32 L = lo[u];
        const i32 nch = (L + CB_THREADS - 1) / CB_THREADS;
        auto run_of = [&](i32 k, i64& s0, i32& len) {
            len = rpos[b + k];  // neighbours of the middle below u: the first rpos entries of its row
            s0 = mir[b + k] - len;
        };
        // pass A: count the wedge ends
        i32 T = 0;
        for (i32 ch = 0; ch < nch; ++ch) {
            T = flatten_runs(L, ch * CB_THREADS, run_of, R);
            i32 ta, tb;
            wave_share(T, ta, tb);
            run_walk<4>(ta, tb, R.rbase, R.rstart, R.nruns, R.flags[threadIdx.x / WAVE], ridx,
                        [&](bool act, i32, i32, i32 w, i64, u64, i32) {
                            if (act) c4h_add(tab, w, cb);
                        });
            __syncthreads();
        }
        // pass C: c - 1 to the middle of every wedge (one chunk: its runs are still in LDS)
        for (i32 ch = 0; ch < nch; ++ch) {
            if (nch > 1) T = flatten_runs(L, ch * CB_THREADS, run_of, R);
            attribute_middles<true>(T, R, ridx, msum, [&](i32 w) { return c4h_get(tab, w, cb); });
            __syncthreads();
            const i32 k = ch * CB_THREADS + (i32)threadIdx.x;
            if (k < L) {
                const i64 m = msum[threadIdx.x];
                if (m) atomicAdd((unsigned long long*)&c4v[ridx[b + k]], (unsigned long long)m);
                msum[threadIdx.x] = 0;
            }
        }
        // pass B: C(c, 2) to every end w and to u (after the gathers, so that
        // these atomics hold back no load of the walks)
        i64 accu = 0;
        for (int q = threadIdx.x; q < C4H_SLOTS; q += CB_THREADS) {
            const u32 e = tab[q];
            const i64 c = e & cmask;
            if (c >= 2) {
                const i64 pr = c * (c - 1) / 2;
                accu += pr;
                atomicAdd((unsigned long long*)&c4v[e >> cb], (unsigned long long)pr);
            }
        }
        accu = wave_sum(accu);
        if (lane_id() == 0 && accu) atomicAdd((unsigned long long*)&red, (unsigned long long)accu);
        __syncthreads();
        for (int q = threadIdx.x; q < C4H_SLOTS; q += CB_THREADS) tab[q] = 0;
        if (threadIdx.x == 0) {
            if (red) atomicAdd((unsigned long long*)&c4v[u], (unsigned long long)red);
            red = 0;
            sj = nxt;
        }
        __syncthreads();
    }
}

// ---- window tier: dense counters for the ranks [W0, W0 + WS) of one window,
// 16-bit halves of 32-bit words when every count fits 16 bits (d_max < 65536).

static constexpr int C4W_WORDS = 32768;  // 128 KiB

template <bool PACK16>
__device__ __forceinline__ void c4w_inc(u32* cnt, i32 x) {
    if (PACK16) atomicAdd(&cnt[x >> 1], 1u << ((x & 1) << 4));
    else atomicAdd(&cnt[x], 1u);
}

template <bool PACK16>
__device__ __forceinline__ u32 c4w_get(const u32* cnt, i32 x) {
    if (PACK16) return (cnt[x >> 1] >> ((x & 1) << 4)) & 0xffffu;
    return cnt[x];
}

// Pass C from the scratch copy of a chunk's wedge ends, words
// (middle << 16) | (end - W0) in middle order at sc[cs .. ce): every end gives
// cnt - 1 to its middle.  Each thread takes a group of 8 consecutive words
// (two 16-byte loads; the scratch slice starts on a 256-byte boundary and
// holds a multiple of 8 words), reads their counts, then sums them along its
// pieces of the middles' runs, one LDS atomic per piece; the next group's
// loads are in flight meanwhile.  Words of a group outside [cs, ce) are read
// but not counted (their low halves still index the counters in range).
__device__ __forceinline__ void c4w_stream_c(const u32* __restrict__ sc, i32 cs, i32 ce, i32 k0, const u32* cnt,
                                             u32* msum) {
    const i32 g1 = (ce + 7) >> 3;
    i32 g = (cs >> 3) + (i32)threadIdx.x;
    if (g >= g1) return;
    auto load = [&](i32 gg, uint4& a, uint4& b) {
        a = *reinterpret_cast<const uint4*>(sc + 8 * (i64)gg);
        b = *reinterpret_cast<const uint4*>(sc + 8 * (i64)gg + 4);
    };
    uint4 qa, qb;
    load(g, qa, qb);
    while (true) {
        // the next group's words are loaded before this group is summed; the
        // last round loads its own group again, so that every round issues
        // the same loads and the compiler need not wait for them early
        const i32 gn = g + CB_THREADS;
        uint4 na, nb;
        load(min(gn, g1 - 1), na, nb);
        const u32 wd[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
        u32 c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = (cnt[(wd[j] & 0xffffu) >> 1] >> ((wd[j] & 1u) << 4)) & 0xffffu;
        const i32 jlo = cs - 8 * g, jhi = ce - 8 * g;  // words j in [jlo, jhi) belong to the chunk
        u32 kc = 0xffffffffu, sum = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < jlo || j >= jhi) continue;
            const u32 k = wd[j] >> 16;
            if (k != kc) {  // a new piece: the previous one's sum goes out
                if (sum) atomicAdd(&msum[kc - (u32)k0], sum);
                kc = k;
                sum = 0;
            }
            sum += c[j] - 1u;
        }
        if (sum) atomicAdd(&msum[kc - (u32)k0], sum);
        if (gn >= g1) break;
        g = gn;
        qa = na;
        qb = nb;
    }
}

// The job a queue ticket t stands for: in order (vertex by vertex, largest
// first, top window first), except for a part of fewer vertices than
// workgroups with 32-bit counters: there, in order, the whole GPU would work on
// the windows of one or two vertices at a time, all adding to the same N-
// entries' middle sums, so a stride of 7919 (prime: a permutation unless it
// divides the job count) spreads the concurrent jobs over the vertices.
// Tickets at or past the end stay as they are.
template <bool PACK16>
__device__ __forceinline__ i64 c4w_job_order(i64 t, i64 njobs, i64 nh) {
    if (PACK16 || nh >= C4W_GRID || t >= njobs || njobs % 7919 == 0) return t;
    return (t * 7919) % njobs;
}

// Windows per job of a vertex with more than one chunk of middles and nw
// windows, in a part of nh vertices: `group` when the middles' run words fit
// (L <= lmax) and the part's windows leave every workgroup several jobs,
// fewer when they do not (a few heavy vertices keep a job per window); a
// negative group is a plan's setting, taken as it is (-group windows).
__device__ __forceinline__ i64 c4w_gsz(i64 group, i64 L, i64 lmax, i64 nw, i64 nh) {
    if ((group <= 1 && group >= -1) || L > lmax) return 1;
    if (group < 0) return -group;  // as the plan sets it
    const i64 g = nw * nh / (8 * C4W_GRID);
    return g < 1 ? 1 : g > group ? group : g;
}

// Jobs: window-tier vertices in descending rank order (hs holds them in
// ascending order); a vertex whose middles fit one chunk is one job over all
// its windows, top window first; a larger one is one job per window.
// TABM: how a middle's run in a window is found -- 0: binary searches of its
// row, 1: the window table of its vertex (tab), 2: the per-entry window table
// (etab, 16-bit counts only: entries below 65536), whose reads for consecutive
// middles are consecutive, 3 (32-bit counts): the 16-bit window table's
// entries on each side of a 32768-rank boundary, then a search between them
// (searches of the whole row for a middle whose cut is 65536 or more).
template <bool PACK16, int TABM>
__global__ void __launch_bounds__(CB_THREADS) k_c4_window(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                          const i32* __restrict__ lo, const i32* __restrict__ rpos,
                                                          const i64* __restrict__ mir,
                                                          const i32* __restrict__ tab, i64 TS,
                                                          const u16* __restrict__ etab, const i64* __restrict__ ebase,
                                                          const i32* __restrict__ hs_all, const DevPlan* __restrict__ plan,
                                                          const i64* __restrict__ jobpre, u32* __restrict__ job_ctr,
                                                          u32* __restrict__ scr, i64 scr_cap, int etab_mode,
                                                          i32 group, i64 lmax,
                                                          i64* __restrict__ esum, i64* __restrict__ c4v) {
    constexpr i32 WS = PACK16 ? 2 * C4W_WORDS : C4W_WORDS;
    // the part of the window list this launch takes (16-bit counters: the
    // first ranks, 32-bit: the last), and its first window, from the device plan
    FGLT_GATE(&plan->err);
    if (etab_mode == 2 && !plan->use_etab) return;
    if (etab_mode == 1 && plan->use_etab) return;
    const u32 c3 = plan->n_c4[3];
    const u32 nheavy = plan->n_c4_heavy < c3 ? plan->n_c4_heavy : c3;
    const u32 nh = PACK16 ? c3 - nheavy : nheavy;
    const i32* const hs = PACK16 ? hs_all : hs_all + (c3 - nheavy);
    const i32 wlo = (i32)(plan->n_low / WS);
    if (nh == 0) return;
    constexpr bool TAB = TABM == 1 || TABM == 2, ETAB = TABM == 2;
    static_assert(TABM != 3 || !PACK16, "table brackets serve the 32-bit counters' windows");
    using TabT = std::conditional_t<PACK16, u16, i32>;  // the vertex table's entries
    const TabT* const tabt = reinterpret_cast<const TabT*>(tab);
    static_assert(!ETAB || PACK16, "the per-entry table holds 16-bit entries");
    constexpr int MAXCH = 64;  // chunks of a vertex: |N-(u)| < 65536 when counts are packed
    __shared__ u32 cnt[C4W_WORDS];
    __shared__ RunLds R;
    // middles' sums: with 16-bit counts a middle's sum stays below 2^32 (per
    // window: at most 2^16 ends times counts below 2^16; over all windows of a
    // one-chunk job: degree below 2^21 times counts below 2^10)
    // With a scratch copy (16-bit counts), two buffers by chunk parity: a
    // chunk's flush (each thread reads and clears its own entry) may still run
    // while faster wavefronts stream the next chunk, which has no barrier
    // before its atomics; the flush of that next chunk begins with one, so the
    // chunk after it may reuse the buffer.  Gathered chunks start with a
    // barrier of their own.
    using MS = std::conditional_t<PACK16, u32, i64>;
    constexpr int NMS = PACK16 ? 2 : 1;
    __shared__ MS msum[NMS * CB_THREADS];
    __shared__ i32 cst[MAXCH + 1];  // scratch offset of each chunk's ends (pass A order)
    u32* const sc = scr + (i64)blockIdx.x * scr_cap;
    // the last 64 words of the slice are a sink that nobody reads.  Grouped
    // windows (runs searched or bracketed by the 16-bit table, vertices of at
    // most lmax middles) keep each
    // middle's run in the current window in the slice: with 16-bit counts one
    // word per middle before the sink, start (back from the middle's row
    // cut) | length << 16, both below 2^16; with 32-bit counts (no copy of
    // the ends) two words per middle from the slice's start
    const bool grouped = (TABM == 0 || TABM == 3) && (group > 1 || group < -1);
    const i64 scr_use = scr_cap - WAVE - (grouped && PACK16 ? lmax : 0);
    const u32 sink = (u32)(scr_cap - WAVE + lane_id());
    u32* const runw = PACK16 ? sc + scr_use : sc;
    __shared__ i64 sj, sh, red;
    const int wv = threadIdx.x / WAVE, l = lane_id();
    const i64 njobs = jobpre[nh];
    for (int q = threadIdx.x; q < C4W_WORDS; q += CB_THREADS) cnt[q] = 0;
    for (int q = threadIdx.x; q < NMS * CB_THREADS; q += CB_THREADS) msum[q] = 0;
    if (wv == 0) {
        i64 j = 0;
        if (l == 0) j = atomicAdd(job_ctr, 1u);
        j = __shfl(j, 0, WAVE);
        j = c4w_job_order<PACK16>(j, njobs, nh);
        const i64 h = j < njobs ? wave_last_le(jobpre, nh, j) : 0;
        if (l == 0) {
            sj = j;
            sh = h;
            red = 0;
        }
    }
    __syncthreads();
    while (true) {
        const i64 j = sj, h = sh;
        if (j >= njobs) break;
        u32 nxt = 0;
        if (threadIdx.x == 0) nxt = atomicAdd(job_ctr, 1u);  // consumed at the end of this job
        const i32 u = hs[nh - 1 - h];
        const i64 b = roff[u];
        const i32 L = lo[u];
        const i32 nwin = (i32)(((i64)u + WS - 1) / WS);
        const bool single = L <= CB_THREADS;
        const i32 nch = single ? 1 : (L + CB_THREADS - 1) / CB_THREADS;
        // windows below wlo hold only ranks of degree <= 1: every count there
        // is at most 1 and adds nothing, so they are not visited
        // a larger vertex: several windows per job when grouped (c4w_gsz),
        // with its middles' run words kept between them
        const i32 gsz = grouped && !single ? (i32)c4w_gsz(group, L, lmax, nwin - wlo, nh) : 1;
        const bool grp = gsz > 1;
        const i32 wtop = single ? nwin - 1 : nwin - 1 - gsz * (i32)(j - jobpre[h]);
        const i32 wbot = single ? wlo : (wtop - gsz + 1 > wlo ? wtop - gsz + 1 : wlo);
        const i64 eb = ETAB ? ebase[nh - 1 - h] : 0;  // this vertex's block of etab: [window][middle]
        // one chunk: thread k keeps middle k and the end of its not yet
        // visited run (windows go top-down, so each run ends where the
        // previous window's run began); its LDS sum msum[k] collects the
        // middle's share over all windows
        // (with the window table, the table entry of the next window is loaded
        // one window ahead)
        i32 mv = 0, mcut = 0, tcur = 0, tnx = 0;
        i64 mrs = 0, mhi = 0;
        if (single && (i32)threadIdx.x < L) {
            mv = ridx[b + threadIdx.x];
            mcut = rpos[b + threadIdx.x];
            mrs = mir[b + threadIdx.x] - mcut;
            mhi = mrs + mcut;
            if (TAB) tcur = ETAB ? (i32)etab[eb + (i64)wtop * L + threadIdx.x] : (i32)tabt[(i64)mv * TS + wtop];
        }
        // more than one chunk: pass A loads the row data of the next chunk's
        // middles (rpos, mir, and ridx or their etab entries) while it walks
        // the current chunk
        i32 pc_cut = 0, pc_v = 0, pn_cut = 0, pn_v = 0, pc_a1 = 0, pn_a1 = 0;
        i64 pc_mir = 0, pn_mir = 0;
        bool prefetched = false;  // run_of takes the loaded values (pass A), else loads them
        i64 accu = 0;
        for (i32 win = wtop; win >= wbot; --win, tcur = tnx) {
            if (TAB && single && (i32)threadIdx.x < L && win > wbot)
                tnx = ETAB ? (i32)etab[eb + (i64)(win - 1) * L + threadIdx.x] : (i32)tabt[(i64)mv * TS + win - 1];
            const i32 W0 = win * WS;
            const i32 W1 = (i32)std::min<i64>((i64)W0 + WS, u);
            auto run_of = [&](i32 k, i64& s0, i32& len) {
                if (single) {
                    const i64 a0 = TAB ? mrs + (ETAB ? tcur : std::min(tcur, mcut)) : lower_bound_back(ridx, mrs, mhi, W0);
                    s0 = a0;
                    len = (i32)(mhi - a0);
                    mhi = a0;
                } else {
                    const i32 cut = prefetched ? pc_cut : rpos[b + k];
                    const i64 rs = (prefetched ? pc_mir : mir[b + k]) - cut;
                    if (ETAB) {  // entries already clamped to the cut
                        const i32 a0 = prefetched ? pc_v : (i32)etab[eb + (i64)win * L + k];
                        const i32 a1 = prefetched ? pc_a1 : (i32)etab[eb + (i64)(win + 1) * L + k];
                        s0 = rs + a0;
                        len = a1 - a0;
                    } else if (TAB) {
                        const i64 vrow = (i64)(prefetched ? pc_v : ridx[b + k]) * TS;
                        const i32 a0 = std::min((i32)tabt[vrow + win], cut);
                        const i32 a1 = std::min((i32)tabt[vrow + win + 1], cut);
                        s0 = rs + a0;
                        len = a1 - a0;
                    } else if (grp) {
                        // pass A (the loaded values): the run ends where the
                        // previous window's run began (a search of the row for
                        // the job's top window), and its start comes by
                        // galloping back from there; pass C reads what pass A
                        // stored (same thread, same k)
                        const i64 re = rs + cut;
                        if (!prefetched) {
                            if (PACK16) {
                                const u32 rw = runw[k];
                                s0 = re - (i64)(rw & 0xffffu);
                                len = (i32)(rw >> 16);
                            } else {
                                s0 = re - (i64)runw[2 * k];
                                len = (i32)runw[2 * k + 1];
                            }
                        } else {
                            const i64 back = win == wtop ? 0 : PACK16 ? (i64)(runw[k] & 0xffffu) : (i64)runw[2 * k];
                            const i64 e = win == wtop ? lower_bound_dev(ridx, rs, re, W1) : re - back;
                            s0 = lower_bound_back(ridx, rs, e, W0);
                            len = (i32)(e - s0);
                            if (PACK16) {
                                runw[k] = (u32)(re - s0) | ((u32)len << 16);
                            } else {
                                runw[2 * k] = (u32)(re - s0);
                                runw[2 * k + 1] = (u32)len;
                            }
                        }
                    } else if (TABM == 3 && cut < 65536) {
                        // the 16-bit vertex table brackets a 32768-rank window
                        // boundary between two 65536-rank ones: below u every
                        // count is at most the cut, so the entries hold
                        const i64 re = rs + cut;
                        const u16* const t16 =
                            reinterpret_cast<const u16*>(tab) + (i64)(prefetched ? pc_v : ridx[b + k]) * TS;
                        auto pos_of = [&](i32 W) -> i64 {  // first entry of the row at rank >= W
                            if (W >= u) return re;
                            const i32 q = W >> 16;
                            const i64 p0 = rs + t16[q];
                            if ((W & 0xffff) == 0) return p0;
                            const i64 p1 = ((i64)(q + 1) << 16) >= u ? re : rs + t16[q + 1];
                            return lower_bound_dev(ridx, p0, p1, W);
                        };
                        s0 = pos_of(W0);
                        len = (i32)(pos_of(W1) - s0);
                    } else {
                        const i64 re = rs + cut;
                        s0 = lower_bound_dev(ridx, rs, re, W0);
                        len = (i32)(lower_bound_fwd(ridx, s0, re, W1) - s0);
                    }
                }
            };
            // pass A: count the wedge ends inside the window; with packed
            // counts, also copy the ends with their middles to the
            // workgroup's scratch (chunk by chunk while they fit), so that
            // pass C streams them instead of gathering the rows again
            i32 T = 0;
            i64 wtot = 0;     // wedges of the window (block-uniform)
            i64 toff = 0;     // scratch words used (block-uniform)
            u64 stored = 0;   // chunks whose ends are in the scratch
            prefetched = !single;
            for (i32 ch = 0; ch < nch; ++ch) {
                if (!single) {
                    const i32 k = ch * CB_THREADS + (i32)threadIdx.x;
                    if (ch == 0 && k < L) {
                        pn_cut = rpos[b + k];
                        pn_mir = mir[b + k];
                        if (ETAB) {
                            pn_v = etab[eb + (i64)win * L + k];
                            pn_a1 = etab[eb + (i64)(win + 1) * L + k];
                        } else {
                            pn_v = ridx[b + k];
                        }
                    }
                    pc_cut = pn_cut;
                    pc_mir = pn_mir;
                    pc_v = pn_v;
                    pc_a1 = pn_a1;
                }
                T = flatten_runs(L, ch * CB_THREADS, run_of, R);
                if (!single && ch + 1 < nch) {
                    const i32 k = (ch + 1) * CB_THREADS + (i32)threadIdx.x;
                    if (k < L) {
                        pn_cut = rpos[b + k];
                        pn_mir = mir[b + k];
                        if (ETAB) {
                            pn_v = etab[eb + (i64)win * L + k];
                            pn_a1 = etab[eb + (i64)(win + 1) * L + k];
                        } else {
                            pn_v = ridx[b + k];
                        }
                    }
                }
                const bool keep = PACK16 && ch < MAXCH && toff + T <= scr_use;
                if (keep && threadIdx.x == 0) {
                    cst[ch] = (i32)toff;
                    cst[ch + 1] = (i32)(toff + T);
                }
                const i32 k0 = ch * CB_THREADS;
                i32 ta, tb;
                wave_share(T, ta, tb);
                // every lane stores its word, an item that is not copied to the
                // sink: the walk keeps the next gathers in flight only where
                // its stores do not depend on the path.  32-bit byte offsets
                // from the slice (below 2^22).
                char* const scb = reinterpret_cast<char*>(sc);
                run_walk_pipe<4>(ta, tb, R.rbase, R.rstart, R.rk, R.nruns, R.flags[wv], ridx,
                                 [&](bool act, i32 t, i32 kr, i32 w) {
                                     if (act) c4w_inc<PACK16>(cnt, w - W0);
                                     const u32 word = ((u32)(k0 + kr) << 16) | (u32)(w - W0);
                                     const u32 off = act && keep ? (u32)toff + (u32)t : sink;
                                     *reinterpret_cast<u32*>(scb + (off << 2)) = word;
                                 });
                if (keep) {
                    stored |= 1ull << ch;
                    toff += T;
                }
                wtot += T;
                if (!single) __syncthreads();  // the next chunk overwrites the runs
            }
            __syncthreads();
            if (wtot == 0) continue;  // no wedge in this window (block-uniform)
            // pass C: c - 1 to the middle of every wedge, streamed from the
            // scratch, else gathered again (one chunk: its runs are still in LDS)
            prefetched = false;
            for (i32 ch = 0; ch < nch; ++ch) {
                MS* const ms = msum + (ch % NMS) * CB_THREADS;
                bool streamed = false;
                if constexpr (PACK16) {  // only 16-bit counters keep a scratch copy
                    if ((stored >> ch) & 1ull) {
                        c4w_stream_c(sc, cst[ch], cst[ch + 1], ch * CB_THREADS, cnt, ms);
                        streamed = true;
                    }
                }
                if (!streamed) {
                    if (!single) T = flatten_runs(L, ch * CB_THREADS, run_of, R);
                    attribute_middles<PACK16>(T, R, ridx, ms,
                                              [&](i32 w) { return c4w_get<PACK16>(cnt, w - W0); });
                }
                if (!single) {
                    // the chunk's middle sums go to their N- entries of u:
                    // consecutive words, so a wavefront's atomics share a few
                    // cache lines; every window of u adds to the same entries,
                    // and k_c4_esum_flush moves them to the middles at the end
                    __syncthreads();
                    const i32 k = ch * CB_THREADS + (i32)threadIdx.x;
                    if (k < L) {
                        const i64 m = ms[threadIdx.x];
                        if (m) atomicAdd((unsigned long long*)&esum[b + k], (unsigned long long)m);
                        ms[threadIdx.x] = 0;
                    }
                }
            }
            // pass B: C(c, 2) to every end w and to u (after the gathers, so
            // that these atomics hold back no load of the walks).  A window
            // with fewer wedges than twice its counter words goes over the
            // scratch copy of its wedges: the first wedge of each end takes the
            // end's count and clears it, which also leaves the counters zero
            // for the next window.  Otherwise the counters are read word by
            // word, then cleared.
            const bool all_kept = nch <= MAXCH && stored == (nch == 64 ? ~0ull : ((1ull << nch) - 1));
            const bool sparse = PACK16 && all_kept && toff < 2 * (i64)C4W_WORDS;
            if (sparse) {
                __syncthreads();  // every count has been read by pass C
                // four words in flight per thread: a load waits for the global
                // atomics issued before it, so the loads go first
                for (i32 t0 = (i32)threadIdx.x; t0 < (i32)toff; t0 += 4 * CB_THREADS) {
                    u32 xv[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const i32 t = t0 + q * CB_THREADS;
                        xv[q] = t < (i32)toff ? sc[t] & 0xffffu : 0xffffffffu;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (xv[q] == 0xffffffffu) continue;
                        const u32 x = xv[q];
                        const u32 sh = (x & 1u) << 4;
                        const u32 old = atomicAnd(&cnt[x >> 1], ~(0xffffu << sh));
                        const i64 c = (old >> sh) & 0xffffu;
                        if (c >= 2) {
                            const i64 pr = c * (c - 1) / 2;
                            accu += pr;
                            atomicAdd((unsigned long long*)&c4v[W0 + x], (unsigned long long)pr);
                        }
                    }
                }
            } else if (PACK16) {  // word by word: two counts per word, most words zero
                for (i32 q = (i32)threadIdx.x; q < C4W_WORDS; q += CB_THREADS) {
                    const u32 wd = cnt[q];
                    if (wd == 0) continue;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const i64 c = (wd >> (16 * h)) & 0xffffu;
                        if (c >= 2) {
                            const i64 pr = c * (c - 1) / 2;
                            accu += pr;
                            atomicAdd((unsigned long long*)&c4v[W0 + 2 * q + h], (unsigned long long)pr);
                        }
                    }
                }
            } else {
                for (i32 x = (i32)threadIdx.x; x < C4W_WORDS; x += CB_THREADS) {
                    const i64 c = c4w_get<PACK16>(cnt, x);
                    if (c >= 2) {
                        const i64 pr = c * (c - 1) / 2;
                        accu += pr;
                        atomicAdd((unsigned long long*)&c4v[W0 + x], (unsigned long long)pr);
                    }
                }
            }
            __syncthreads();
            if (!sparse) {  // clear the counters for the next window
                for (i32 q = (i32)threadIdx.x; q < C4W_WORDS; q += CB_THREADS) cnt[q] = 0;
            }
        }
        accu = wave_sum(accu);
        if (l == 0 && accu) atomicAdd((unsigned long long*)&red, (unsigned long long)accu);
        __syncthreads();
        if (single && (i32)threadIdx.x < L) {
            const i64 m = msum[threadIdx.x];
            if (m) atomicAdd((unsigned long long*)&c4v[mv], (unsigned long long)m);
            msum[threadIdx.x] = 0;
        }
        if (threadIdx.x == 0) {
            if (red) atomicAdd((unsigned long long*)&c4v[u], (unsigned long long)red);
            red = 0;
        }
        if (wv == 0) {  // decode the next job
            const i64 nj = c4w_job_order<PACK16>(__shfl((i64)nxt, 0, WAVE), njobs, nh);
            const i64 nhh = nj < njobs ? wave_last_le(jobpre, nh, nj) : 0;
            if (l == 0) {
                sj = nj;
                sh = nhh;
            }
        }
        __syncthreads();
    }
}

// The middle sums that the window kernels left per N- entry (vertices whose
// middles span several chunks, one job per window) go to the middles: one
// streaming pass over the entries, an atomic for each non-zero sum.
__global__ void k_c4_esum_flush(const i32* __restrict__ ridx, const i64* __restrict__ esum, i64 nnz,
                                i64* __restrict__ c4v, const DevPlan* __restrict__ plan) {
    FGLT_GATE(&plan->err);
    if (plan->n_c4[3] == 0) return;
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (i64)gridDim.x * blockDim.x) {
        const i64 m = esum[q];
        if (m) atomicAdd((unsigned long long*)&c4v[ridx[q]], (unsigned long long)m);
    }
}

// The window list's part of one counter width (heavy: 32-bit counters, the
// last nheavy entries of the ascending list), from the device plan.
__device__ __forceinline__ void c4w_part(const DevPlan* plan, const i32* hs_all, bool heavy, const i32*& hs, u32& nh) {
    const u32 c3 = plan->n_c4[3];
    const u32 nheavy = plan->n_c4_heavy < c3 ? plan->n_c4_heavy : c3;
    nh = heavy ? nheavy : c3 - nheavy;
    hs = heavy ? hs_all + (c3 - nheavy) : hs_all;
}

// Window table: tab[v * TS + k] = number of neighbours of v with rank below
// k * WS, for k < K1; rows of TS entries start on 32-byte boundaries.  T is
// u16 where every degree is below 65536, else i32.
template <class T>
__global__ void k_c4_table(const i64* __restrict__ roff, const i32* __restrict__ ridx, i64 n, i64 K1, i64 TS, i64 WS,
                           T* __restrict__ tab, const DevPlan* __restrict__ plan) {
    FGLT_GATE(&plan->err);
    if (plan->n_c4[3] == 0) return;  // no window job
    const i64 total = n * K1;
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (i64)gridDim.x * blockDim.x) {
        const i64 v = q / K1, k = q - v * K1;
        const i64 b = roff[v], e = roff[v + 1];
        const i64 key = k * WS;
        tab[v * TS + k] = (T)(key >= n ? e - b : lower_bound_dev(ridx, b, e, key) - b);
    }
}

// Per-entry window table, sizes: the i-th window-tier vertex u (hs in
// ascending order) has L = |N-(u)| middles and ceil(u / WS) windows; its
// block holds one entry per middle and window boundary, and its middles
// make ceil(L / ET_CHUNK) chunks of the build.
static constexpr int ET_CHUNK = 256;

__global__ void k_c4_ecount(const i32* __restrict__ hs_all, const i32* __restrict__ lo,
                            const DevPlan* __restrict__ plan, i64 WS, i64 bound, i64* __restrict__ ecnt,
                            i64* __restrict__ ccnt) {
    FGLT_GATE(&plan->err);
    const i32* hs;
    u32 nh;
    c4w_part(plan, hs_all, false, hs, nh);
    if (!plan->use_etab) nh = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < bound; i += (i64)gridDim.x * blockDim.x) {
        const i64 u = i < (i64)nh ? hs[i] : 0;
        ecnt[i] = i < (i64)nh ? (i64)lo[u] * ((u + WS - 1) / WS + 1) : 0;
        ccnt[i] = i < (i64)nh ? ((i64)lo[u] + ET_CHUNK - 1) / ET_CHUNK : 0;
    }
}

// Per-entry window table: etab[ebase[i] + w * L + k] = the position in the
// row of middle k (the k-th lower neighbour of u, the i-th window-tier
// vertex) of its first neighbour of rank >= w * WS, at most its cut (the
// position of u).  With 16-bit counts every row is shorter than 65536.  A
// workgroup per chunk of ET_CHUNK middles (cpre: prefix of the chunk counts;
// wavefront 0 finds the chunk's vertex); a thread reads its middle's row of
// the 16-bit vertex table (row stride TS) with 16-byte loads and writes one
// entry per window, consecutive across the threads.
__global__ void __launch_bounds__(ET_CHUNK) k_c4_etab(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                      const i32* __restrict__ lo, const i32* __restrict__ rpos,
                                                      const u16* __restrict__ tab, i64 TS,
                                                      const i32* __restrict__ hs_all, const DevPlan* __restrict__ plan,
                                                      const i64* __restrict__ cpre, const i64* __restrict__ ebase,
                                                      i64 WS, u16* __restrict__ etab) {
    FGLT_GATE(&plan->err);
    if (!plan->use_etab) return;
    const i32* hs;
    u32 nh;
    c4w_part(plan, hs_all, false, hs, nh);
    __shared__ i64 si;
    const i64 nchunks = cpre[nh];
    for (i64 c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (threadIdx.x < WAVE) {
            const i64 i = wave_last_le(cpre, nh, c);  // cpre[i] <= c < cpre[i + 1]
            if (threadIdx.x == 0) si = i;
        }
        __syncthreads();
        const i64 i = si;
        const i64 u = hs[i];
        const i64 L = lo[u];
        const i64 k = (c - cpre[i]) * ET_CHUNK + threadIdx.x;
        if (k < L) {
            const i32 nwin = (i32)((u + WS - 1) / WS);
            const i64 b = roff[u];
            const i64 vrow = (i64)ridx[b + k] * TS;
            const i32 cut = rpos[b + k];
            u16* const out = etab + ebase[i] + k;
            // 16-byte loads of 8 entries: the row starts on a 32-byte boundary
            // and holds a multiple of 16 entries, so entries w0 .. w0 + 7 are inside it
            const uint4* const row = reinterpret_cast<const uint4*>(tab + vrow);
            for (i32 w0 = 0; w0 <= nwin; w0 += 8) {
                const uint4 x = row[w0 / 8];
                const i32 v[8] = {(i32)(x.x & 0xffffu), (i32)(x.x >> 16), (i32)(x.y & 0xffffu), (i32)(x.y >> 16),
                                  (i32)(x.z & 0xffffu), (i32)(x.z >> 16), (i32)(x.w & 0xffffu), (i32)(x.w >> 16)};
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (w0 + q <= nwin) out[(i64)(w0 + q) * L] = (u16)std::min(v[q], cut);
            }
        }
        __syncthreads();  // si is rewritten by the next chunk
    }
}

// The one segment of the window-tier list's sort: [0, its size).
__global__ void k_c4_segment(i64* p, const DevPlan* __restrict__ plan) {
    p[0] = 0;
    p[1] = plan->err ? 0 : plan->n_c4[3];
}

// Jobs per window-tier vertex of one part, in descending vertex order: one
// over windows wlo .. ceil(u / WS) - 1 for a vertex whose middles fit one
// chunk, else one per window (none when no window is left); zero from the
// part's size up to `bound`, so that the prefix over `bound` entries holds.
__global__ void k_c4_jobs(const i32* __restrict__ hs_all, const i32* __restrict__ lo, const DevPlan* __restrict__ plan,
                          int heavy, i64 WS, i64 group, i64 lmax, i64 bound, i64* __restrict__ jobcnt) {
    FGLT_GATE(&plan->err);
    const i32* hs;
    u32 nh;
    c4w_part(plan, hs_all, heavy != 0, hs, nh);
    const i64 wlo = plan->n_low / WS;
    for (i64 h = (i64)blockIdx.x * blockDim.x + threadIdx.x; h < bound; h += (i64)gridDim.x * blockDim.x) {
        i64 c = 0;
        if (h < (i64)nh) {
            const i64 u = hs[nh - 1 - h];
            const i64 nw = std::max<i64>(0, (u + WS - 1) / WS - wlo);
            const i64 g = c4w_gsz(group, lo[u], lmax, nw, nh);  // as the window kernel groups them
            c = lo[u] <= CB_THREADS ? std::min<i64>(nw, 1) : (nw + g - 1) / g;
        }
        jobcnt[h] = c;
    }
}

// ------------------------------------------------------------ launcher

// The window tier's configuration, the same in every part of the pass.  The
// tier's vertices (ascending rank) split into those of degree below 65536 --
// every count and every middle's row position fits 16 bits, since a middle
// ranks below its vertex and so has no larger degree -- counted with 16-bit
// counters over 65536-rank windows, and the rest (the last ranks), counted
// with 32-bit counters over 32768-rank windows and binary searches of the
// middles' rows.  The split, the first window (windows holding only ranks of
// degree <= 1 are skipped) and whether the per-entry table fits are read on
// the device from the plan; the host knows only the sizes.
struct C4WinCfg {
    bool use_tab, want_etab;
    i64 K1, TS;          // the 16-bit vertex table: entries per row, row stride
    i64 bound_l, bound_h;  // entries of the job arrays of each part (at least its size)
    // windows per job of a vertex with more than one chunk of middles and at
    // most lmax of them, whose run words the scratch slice holds: 16-bit
    // counters with searched runs (no table), one word per middle for up to
    // min(65536, n) middles, when three quarters of the slice stay for the
    // wedge ends; 32-bit counters (searched or bracketed runs, no copy of the
    // ends), two words per middle
    i64 group, hgroup, lmax16, lmax32;
};

static constexpr i64 C4W_WS16 = 2 * C4W_WORDS;  // ranks per window, 16-bit counters
static constexpr i64 C4W_WS32 = C4W_WORDS;      // ranks per window, 32-bit counters

static C4WinCfg c4_win_cfg(i64 n, i64 nnz, const RawWs& w, int rows_mode, int win_group) {
    C4WinCfg c;
    c.K1 = (n + C4W_WS16 - 1) / C4W_WS16 + 1;
    // the table's row stride: 32 bytes' worth of entries
    c.TS = (c.K1 + 15) & ~(i64)15;
    c.use_tab = rows_mode != 2 && w.c4_tab != nullptr && n * c.TS <= w.c4_tab_cap;
    // the per-entry window table lives in the stored bitmaps' memory (16-bit
    // entries, four per word); whether it fits is decided on the device
    c.want_etab = rows_mode == 0 && c.use_tab;
    c.bound_l = n;
    c.bound_h = std::min<i64>(n, (nnz >> 16) + 1);  // vertices of degree >= 65536
    // a plan's group is taken as it is (negative: exactly that many), the
    // default adapts to the part's size (c4w_gsz)
    const i64 g = win_group > 0 ? -(i64)win_group : C4W_GROUP;
    c.group = c.use_tab ? 1 : g;
    c.hgroup = g;  // 32-bit counters: runs searched or bracketed, grouped either way
    const i64 m16 = std::min<i64>(65536, std::max<i64>(n, 1));
    c.lmax16 = w.c4_scr_cap >= 4 * m16 + WAVE ? m16 : 0;
    c.lmax32 = (w.c4_scr_cap - WAVE) / 2;
    static_assert(C4W_WS16 == C4W_SPAN, "the tier assignment sizes the table with this window");
    return c;
}

// Part one of the 4-cycle pass: the three hash tiers, then the window tier's
// setup (its vertex list sorted, the vertex table, the job lists, the
// per-entry table's offsets).  It reads only the structure and writes only
// 4-cycle state (the sums, lists, tables, job arrays, and a sort buffer of its
// own), so it may run on a second stream beside the triangle and clique
// passes.  Tier sizes come from the device plan: the grids are bounds.
hipError_t launch_c4_early(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s) {
    hipError_t e;
    if ((e = fill_u32(w.c4_jobctr, 3, 0u, s)) != hipSuccess) return e;
    const u32* const cnt = w.plan->n_c4;
    hipLaunchKernelGGL((k_c4_hash<1, 256>), dim3(grid_for(n, 4, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.lo, w.G,
                       w.mir, w.c4_list, cnt + 0, w.c4v);
    hipLaunchKernelGGL((k_c4_hash<4, 4096>), dim3(grid_for(n, 1, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.lo, w.G,
                       w.mir, w.c4_list + n, cnt + 1, w.c4v);
    {
        const int cb = 32 - std::max(1, bits_for_n(n));
        hipLaunchKernelGGL(k_c4_hashbig, dim3(grid_for(n, 1, 512)), dim3(CB_THREADS), 0, s, w.roff, w.ridx, w.lo,
                           w.rpos, w.mir, w.c4_list + 2 * n, cnt + 2, w.c4_jobctr + 1, cb, w.c4v);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const C4WinCfg c = c4_win_cfg(n, nnz, w, rows_mode, win_group);
    // window-tier vertices in ascending order (the sort's buffer: c4_ebase,
    // not yet in use; the shared one is the clique pass's memory); the
    // vertices of degree >= 65536 end the list
    i32* hs = w.c4_list + 3 * n;
    hipLaunchKernelGGL(k_c4_segment, dim3(1), dim3(1), 0, s, w.c4_segoff, (const DevPlan*)w.plan);
    SegSortWs ws = w.sort;
    ws.tmp = reinterpret_cast<i32*>(w.c4_ebase);
    if ((e = seg_sort(hs, w.c4_segoff, 1, bits_for_n(n), ws, 1, s)) != hipSuccess) return e;
    if (c.use_tab)
        hipLaunchKernelGGL(k_c4_table<u16>, dim3(grid_for(n * c.K1, PT, 65536)), dim3(PT), 0, s, w.roff, w.ridx, n,
                           c.K1, c.TS, C4W_WS16, w.c4_tab, (const DevPlan*)w.plan);
    hipLaunchKernelGGL(k_c4_jobs, dim3(grid_for(c.bound_l, PT, 4096)), dim3(PT), 0, s, hs, w.lo,
                       (const DevPlan*)w.plan, 0, C4W_WS16, c.group, c.lmax16, c.bound_l, w.c4_jobcnt);
    if ((e = scan_exclusive_i64(w.c4_jobcnt, w.c4_jobpre, c.bound_l, w.partials, s)) != hipSuccess) return e;
    if (c.want_etab) {
        // c4_jobcnt is free again once the job prefix is built: the chunk counts
        hipLaunchKernelGGL(k_c4_ecount, dim3(grid_for(c.bound_l, PT, 4096)), dim3(PT), 0, s, hs, w.lo,
                           (const DevPlan*)w.plan, C4W_WS16, c.bound_l, w.c4_ebase, w.c4_jobcnt);
        if ((e = scan_exclusive_i64(w.c4_ebase, w.c4_ebase, c.bound_l, w.partials, s)) != hipSuccess) return e;
        if ((e = scan_exclusive_i64(w.c4_jobcnt, w.c4_jobcnt, c.bound_l, w.partials, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_c4_jobs, dim3(grid_for(c.bound_h, PT, 4096)), dim3(PT), 0, s, hs, w.lo,
                       (const DevPlan*)w.plan, 1, C4W_WS32, c.hgroup, c.lmax32, c.bound_h, w.c4_hjobcnt);
    if ((e = scan_exclusive_i64(w.c4_hjobcnt, w.c4_hjobpre, c.bound_h, w.partials, s)) != hipSuccess) return e;
    return hipGetLastError();
}

// Part two: the per-entry window table, in the stored bitmaps' memory, so
// after the clique pass (it may run on the second stream beside row pass 2).
hipError_t launch_c4_etab(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s) {
    const C4WinCfg c = c4_win_cfg(n, nnz, w, rows_mode, win_group);
    if (c.want_etab)  // 16 workgroups per CU stride over the chunks (their count is on the device)
        hipLaunchKernelGGL(k_c4_etab, dim3(grid_for(nnz, ET_CHUNK, 4096)), dim3(ET_CHUNK), 0, s, w.roff, w.ridx, w.lo,
                           w.rpos, w.c4_tab, c.TS, w.c4_list + 3 * n, (const DevPlan*)w.plan, w.c4_jobcnt, w.c4_ebase,
                           C4W_WS16, reinterpret_cast<u16*>(w.bstore));
    return hipGetLastError();
}

// Part three: the window kernels, 16-bit counters then 32-bit counters.
hipError_t launch_c4_late(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s, SegTimer& tm) {
    tm.mark(FGLT_SEG_C4_WAVE, s);
    tm.mark(FGLT_SEG_C4_BLOCK, s);
    tm.mark(FGLT_SEG_C4_HASH, s);
    tm.mark(FGLT_SEG_C4_WINDOW, s);  // the segment times the window kernels alone
    const C4WinCfg c = c4_win_cfg(n, nnz, w, rows_mode, win_group);
    const i32* hs = w.c4_list + 3 * n;
    const u16* const etab = reinterpret_cast<const u16*>(w.bstore);
    const i32* const tab = reinterpret_cast<const i32*>(w.c4_tab);
    const DevPlan* const plan = w.plan;
    const unsigned grid = C4W_GRID;  // one workgroup per CU; each owns a scratch slice
    // per-entry middle sums of the multi-chunk jobs (the clique pass's
    // per-entry counts are dead once the row pass has read them)
    if (nnz > 0) {
        hipError_t e = fill_u32(reinterpret_cast<u32*>(w.ek), 2 * nnz, 0u, s);
        if (e != hipSuccess) return e;
    }
#define C4W_LAUNCH(P16, TM, PRE, CTR, EM, GRP, LMAX)                                                               \
    hipLaunchKernelGGL((k_c4_window<P16, TM>), dim3(grid), dim3(CB_THREADS), 0, s, w.roff, w.ridx, w.lo, w.rpos, \
                       w.mir, tab, c.TS, etab, w.c4_ebase, hs, plan, PRE, CTR, w.c4_scr, w.c4_scr_cap, EM,         \
                       (i32)(GRP), (i64)(LMAX), w.ek, w.c4v)
    // the per-entry table where it fits (decided on the device), else the vertex table
    if (c.want_etab) C4W_LAUNCH(true, 2, w.c4_jobpre, w.c4_jobctr, 2, 1, 0);
    if (c.use_tab) C4W_LAUNCH(true, 1, w.c4_jobpre, w.c4_jobctr, c.want_etab ? 1 : 0, 1, 0);
    else C4W_LAUNCH(true, 0, w.c4_jobpre, w.c4_jobctr, 0, c.group, c.lmax16);
    tm.note("c4_window (16-bit counters)", s);
    if (c.use_tab) C4W_LAUNCH(false, 3, w.c4_hjobpre, w.c4_jobctr + 2, 0, c.hgroup, c.lmax32);
    else C4W_LAUNCH(false, 0, w.c4_hjobpre, w.c4_jobctr + 2, 0, c.hgroup, c.lmax32);
#undef C4W_LAUNCH
    if (nnz > 0)
        hipLaunchKernelGGL(k_c4_esum_flush, dim3(grid_for(nnz, PT, 8192)), dim3(PT), 0, s, w.ridx,
                           (const i64*)w.ek, nnz, w.c4v, plan);
    return hipGetLastError();
}

}  // namespace fglt
