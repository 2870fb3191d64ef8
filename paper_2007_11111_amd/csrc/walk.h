// walk.h -- wave and workgroup building blocks shared by the counting kernels:
// block scans, the run walk over flattened work items, and LDS hash tables.
#pragma once

#include "raw.h"

namespace fglt {

// Iterates the set bits of a 64-bit word.
#define FOR_BITS(word, var, body)                 \
    do {                                          \
        u64 fb_w_ = (word);                       \
        while (fb_w_) {                           \
            const int var = __ffsll((long long)fb_w_) - 1; \
            fb_w_ &= fb_w_ - 1;                   \
            body;                                 \
        }                                         \
    } while (0)


// Inclusive prefix sum over the 64 lanes of a wavefront with DPP: shifts by
// 1, 2, 4, 8 within each row of 16 lanes, then the row totals broadcast to
// the rows above (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).
__device__ __forceinline__ i32 wave_incl_scan_i32(i32 x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// The same scan for 64-bit values: both halves move together, the sum carries.
template <int CTRL, int ROWS>
__device__ __forceinline__ i64 dpp_add_i64(i64 x) {
    const u32 lo_ = (u32)__builtin_amdgcn_update_dpp(0, (i32)(u32)x, CTRL, ROWS, 0xf, false);
    const u32 hi_ = (u32)__builtin_amdgcn_update_dpp(0, (i32)(u32)((u64)x >> 32), CTRL, ROWS, 0xf, false);
    return x + (i64)(((u64)hi_ << 32) | lo_);
}
__device__ __forceinline__ i64 wave_incl_scan_i64(i64 x) {
    x = dpp_add_i64<0x111, 0xf>(x);  // row_shr:1
    x = dpp_add_i64<0x112, 0xf>(x);  // row_shr:2
    x = dpp_add_i64<0x114, 0xf>(x);  // row_shr:4
    x = dpp_add_i64<0x118, 0xf>(x);  // row_shr:8
    x = dpp_add_i64<0x142, 0xa>(x);  // row_bcast:15
    x = dpp_add_i64<0x143, 0xc>(x);  // row_bcast:31
    return x;
}

// Exclusive scan of one value per thread over a block of NT threads; returns
// the thread's prefix and writes the block total to *total.  Every thread of
// the block must call it.  Both levels scan with DPP, without LDS round trips.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 8) return (T)wave_incl_scan_i64((i64)x);
    else return (T)wave_incl_scan_i32((i32)x);
}

template <int NT, class T>
__device__ __forceinline__ T block_scan(T v, T* wsum, T* total) {
    constexpr int NWV = NT / WAVE;
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    const T x = wave_incl_scan(v);
    if (l == WAVE - 1) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const T y = wave_incl_scan(threadIdx.x < NWV ? wsum[threadIdx.x] : (T)0);
        if (threadIdx.x < NWV) wsum[threadIdx.x] = y;
        if (threadIdx.x == NWV - 1) *total = y;
    }
    __syncthreads();
    return (wv > 0 ? wsum[wv - 1] : 0) + x - v;
}

// Lanes of one wavefront exchange words through LDS: relaxed atomics at
// wavefront scope keep the compiler from forwarding a lane's own store to its
// later load (another lane may have written in between) while still compiling
// to plain ds_write / ds_read, which a wavefront executes in order.  (A
// volatile pointer would do the former but loses the LDS address space and
// turns into system-coherent flat accesses that wait for every outstanding
// global load.)
__device__ __forceinline__ void lds_put(i32* p, i32 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ i32 lds_get(i32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void lds_put8(u8* p, u8 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ u8 lds_get8(u8* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Last index r in [0, R) with a[r] <= key, for a non-decreasing LDS array
// with a[0] <= key and a key that is the same in every lane: each round the
// 64 lanes probe evenly spaced entries, so R entries take about log64(R)
// dependent LDS reads instead of log2(R).
__device__ __forceinline__ i32 wave_last_le_lds(const i32* a, i32 R, i32 key) {
    i32 lo_ = 0, hi_ = R;  // the answer lies in [lo_, hi_)
    while (hi_ - lo_ > 1) {
        const i32 step = (hi_ - lo_ + WAVE - 1) / WAVE;
        const i32 p = lo_ + lane_id() * step;
        const bool ok = p < hi_ && a[p] <= key;
        const int c = __popcll(__ballot(ok));  // lanes 0 .. c-1 probe entries <= key
        lo_ += (c - 1) * step;
        hi_ = min(hi_, lo_ + step);
    }
    return lo_;
}

// Last index h in [0, cnt) with a[h] <= key, for a non-decreasing a with
// a[0] <= key.  The whole wavefront searches, 64 probes per round, so a list
// of N entries takes about log64(N) dependent loads.
__device__ __forceinline__ i64 wave_last_le(const i64* __restrict__ a, i64 cnt, i64 key) {
    i64 lo_ = 0, hi_ = cnt;  // the answer lies in [lo_, hi_)
    while (hi_ - lo_ > 1) {
        const i64 step = (hi_ - lo_ + WAVE - 1) / WAVE;
        const i64 p = lo_ + (i64)lane_id() * step;
        const bool ok = p < hi_ && a[p] <= key;
        const int c = __popcll(__ballot(ok));  // lanes 0 .. c-1 hold probes <= key
        lo_ += (i64)(c - 1) * step;
        hi_ = min(hi_, lo_ + step);
    }
    return lo_;
}

// The run walk, in groups of up to U steps of 64 items.  A group reads the
// starts of the next 64 runs once (one per lane); it ends before the last of
// them, so every item in it has a known run.  The run starts inside the group
// are marked as bytes in the wavefront's 256-byte flags row (cleared, marked,
// then read back once per step: three LDS round trips per group); the run of
// item ts + l is r0 + (starts in earlier steps) + (starts in [ts, ts + l]).
// The run bases (and, keyed, the run keys) are read on every lane at the run
// index clamped to R, so rbase (and rkey) hold R + 1 entries.  The U gathers
// w = ridx[e] of a group are issued together, then
// f(active, item, run, w, e, run-start mask, group end) runs for each step
// (keyed: the run's key rkey[run] in place of the run).  Inactive lanes
// gather a valid dummy item, so no load is branched.
template <int U, bool KEYED, class F>
__device__ __forceinline__ void run_walk_core(i32 ta, i32 tb, const i64* rbase, const i32* rstart, const i32* rkey,
                                              i32 R, i32* flags, const i32* __restrict__ ridx, F&& f) {
    static_assert(U * WAVE <= (int)(WAVE * sizeof(i32)), "one flag byte per item of a group");
    if (ta >= tb) return;
    const int l = lane_id();
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    u8* const fb = reinterpret_cast<u8*>(flags);
    i32 r0 = __builtin_amdgcn_readfirstlane(wave_last_le_lds(rstart, R, ta));  // run holding item ta
    i32 t0 = ta;
    while (t0 < tb) {
        const i32 j = r0 + 1 + l;
        const i32 sj = rstart[j < R ? j : R];
        const i32 st = j < R ? sj : 0x7fffffff;  // start of run r0 + 1 + l (> t0)
        const i32 t1 = min(min(tb, t0 + U * WAVE), __builtin_amdgcn_readlane(st, WAVE - 1));
        const i64 esafe = rbase[r0] + t0;
        lds_put(&flags[l], 0);
        wave_lds_fence();
        if ((u32)(st - t0) < (u32)(U * WAVE)) lds_put8(&fb[st - t0], 1);
        wave_lds_fence();
        u8 fl[U];
#pragma unroll
        for (int s = 0; s < U; ++s) fl[s] = lds_get8(&fb[s * WAVE + l]);
        wave_lds_fence();
        i32 rr[U], kk[U];
        u64 mm[U];
        i64 ee[U];
        i32 ww[U];
        i32 before = 0;  // run starts in the group's earlier steps
#pragma unroll
        for (int s = 0; s < U; ++s) {
            mm[s] = __ballot(fl[s] != 0);
            rr[s] = r0 + before + __popcll(mm[s] & le);
            before += __popcll(mm[s]);
        }
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 t = t0 + s * WAVE + l;
            const i32 rc = min(rr[s], R);
            const i64 bb = rbase[rc];
            kk[s] = KEYED ? rkey[rc] : rr[s];
            ee[s] = t < t1 ? bb + t : esafe;
        }
#pragma unroll
        for (int s = 0; s < U; ++s) ww[s] = ridx[ee[s]];
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 t = t0 + s * WAVE + l;
            f(t < t1, t, kk[s], ww[s], ee[s], mm[s], t1);
        }
        r0 += __popcll(__ballot(st <= t1));  // the run holding item t1
        t0 = t1;
    }
}

template <int U, class F>
__device__ __forceinline__ void run_walk(i32 ta, i32 tb, const i64* rbase, const i32* rstart, i32 R, i32* flags,
                                         const i32* __restrict__ ridx, F&& f) {
    run_walk_core<U, false>(ta, tb, rbase, rstart, nullptr, R, flags, ridx, f);
}

template <int U, class F>
__device__ __forceinline__ void run_walk_keyed(i32 ta, i32 tb, const i64* rbase, const i32* rstart, const i32* rkey,
                                               i32 R, i32* flags, const i32* __restrict__ ridx, F&& f) {
    run_walk_core<U, true>(ta, tb, rbase, rstart, rkey, R, flags, ridx, f);
}

// The run walk with two groups in flight: the runs of the next group are
// found and its gathers issued before the callbacks of the current group
// run, so that the gathers' latency overlaps the per-item work.  Arguments as
// for run_walk, plus rkey, an LDS array with one key per run that the group
// reads together with the run bases (rbase and rkey hold R + 1 entries);
// ridx[0] must be readable.  The callback
// is f(active, item, key of its run, w).  The overlap holds when the
// callback's vector memory operations do not depend on the path either (the
// compiler counts loads in flight per path and takes the smallest count).
template <int U>
struct WalkGroup {
    i32 t0, t1;  // items [t0, t1), the same in every lane; empty when t0 >= the end
    i32 rr[U];
    i32 kk[U];
    u64 mm[U];
    i64 ee[U];
    i32 ww[U];
};

template <int U>
__device__ __forceinline__ void walk_prep(WalkGroup<U>& G, i32& r0, i32& t0, i32 tb, const i64* rbase,
                                          const i32* rstart, const i32* rkey, i32 R, i32* flags,
                                          const i32* __restrict__ ridx, u64 le) {
    G.t0 = t0;
    G.t1 = t0;
    if (t0 < tb) {
        const int l = lane_id();
        u8* const fb = reinterpret_cast<u8*>(flags);
        const i32 j = r0 + 1 + l;
        const i32 sj = rstart[j < R ? j : R];
        const i32 st = j < R ? sj : 0x7fffffff;
        const i32 t1 = min(min(tb, t0 + U * WAVE), __builtin_amdgcn_readlane(st, WAVE - 1));
        const i64 esafe = rbase[r0] + t0;
        lds_put(&flags[l], 0);
        wave_lds_fence();
        if ((u32)(st - t0) < (u32)(U * WAVE)) lds_put8(&fb[st - t0], 1);
        wave_lds_fence();
        u8 fl[U];
#pragma unroll
        for (int s = 0; s < U; ++s) fl[s] = lds_get8(&fb[s * WAVE + l]);
        wave_lds_fence();
        i32 before = 0;
#pragma unroll
        for (int s = 0; s < U; ++s) {
            G.mm[s] = __ballot(fl[s] != 0);
            G.rr[s] = r0 + before + __popcll(G.mm[s] & le);
            before += __popcll(G.mm[s]);
        }
#pragma unroll
        for (int s = 0; s < U; ++s) {  // read on every lane (run index clamped to R) and then
                                       // selected, so that no read depends on the path
            const i32 t = t0 + s * WAVE + l;
            const i32 rc = min(G.rr[s], R);
            const i64 bb = rbase[rc];
            G.kk[s] = rkey[rc];
            G.ee[s] = t < t1 ? bb + t : esafe;
        }
        G.t1 = t1;
        r0 += __popcll(__ballot(st <= t1));
        t0 = t1;
    } else {  // an empty group still issues its gathers (of entry 0), so that
              // the count of loads in flight does not depend on the path
#pragma unroll
        for (int s = 0; s < U; ++s) {
            G.rr[s] = 0;
            G.kk[s] = 0;
            G.mm[s] = 0;
            G.ee[s] = 0;
        }
    }
#pragma unroll
    for (int s = 0; s < U; ++s) G.ww[s] = ridx[G.ee[s]];
}

template <int U, class F>
__device__ __forceinline__ void walk_items(const WalkGroup<U>& G, F& f) {
    const int l = lane_id();
#pragma unroll
    for (int s = 0; s < U; ++s) {
        const i32 t = G.t0 + s * WAVE + l;
        f(t < G.t1, t, G.kk[s], G.ww[s]);
    }
    // every gather of the group has landed here, also where a step had no
    // active lane: otherwise the compiler, to reuse a gather's register in
    // the next group, waits for every load in flight, the next group's too
#pragma unroll
    for (int s = 0; s < U; ++s) asm volatile("" ::"v"(G.ww[s]));
}

template <int U, class F>
__device__ __forceinline__ void run_walk_pipe(i32 ta, i32 tb, const i64* rbase, const i32* rstart, const i32* rkey,
                                              i32 R, i32* flags, const i32* __restrict__ ridx, F&& f) {
    static_assert(U * WAVE <= (int)(WAVE * sizeof(i32)), "one flag byte per item of a group");
    if (ta >= tb) return;
    const int l = lane_id();
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    i32 r0 = __builtin_amdgcn_readfirstlane(wave_last_le_lds(rstart, R, ta));
    i32 t0 = ta;
    WalkGroup<U> A, B;
    walk_prep(A, r0, t0, tb, rbase, rstart, rkey, R, flags, ridx, le);
    while (true) {
        walk_prep(B, r0, t0, tb, rbase, rstart, rkey, R, flags, ridx, le);
        walk_items(A, f);
        if (B.t0 >= tb) break;
        walk_prep(A, r0, t0, tb, rbase, rstart, rkey, R, flags, ridx, le);
        walk_items(B, f);
        if (A.t0 >= tb) break;
    }
}


// Runs of equal keys among the active lanes of a wavefront (active lanes
// first, keys non-decreasing): `tail` on the last lane of each run, `h` the
// first lane of the run holding this lane.  run_total(v) gives every lane the
// sum of v over its run up to itself -- the run's total on its tail lane --
// from one prefix sum and one shuffle from the lane before the run's head.
struct WaveRuns {
    int h;
    bool tail;
};
__device__ __forceinline__ WaveRuns wave_runs(i32 key, bool act) {
    const int l = lane_id();
    const i32 kp = __builtin_amdgcn_update_dpp(0, key, 0x138, 0xf, 0xf, false);  // wave_shr:1
    const i32 kn = __builtin_amdgcn_update_dpp(0, key, 0x130, 0xf, 0xf, false);  // wave_shl:1
    const u64 am = __ballot(act);
    const u64 hm = __ballot(act && (l == 0 || kp != key));
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    const u64 below = hm & le;
    WaveRuns w;
    w.h = below ? 63 - __clzll((long long)below) : 0;
    w.tail = act && (l == WAVE - 1 || kn != key || !((am >> (l + 1)) & 1ull));
    return w;
}
__device__ __forceinline__ i64 run_total(i64 v, const WaveRuns& w) {
    const i64 P = wave_incl_scan_i64(v);
    const i64 Pb = __shfl(P, w.h > 0 ? w.h - 1 : 0, WAVE);
    return w.h > 0 ? P - Pb : P;
}

// Transpose of a 64 x 64 bit matrix held one row per lane (bit j of lane i's
// word = entry (i, j)): returns column `lane`.  Six butterfly rounds; round s
// swaps the off-diagonal s x s blocks of every 2s x 2s block.
__device__ __forceinline__ u64 wave_transpose64(u64 m) {
    const int l = lane_id();
    const u64 M0[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                       0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int r = 0; r < 6; ++r) {
        const int s = 32 >> r;
        const u64 p = __shfl_xor(m, s, WAVE);
        m = (l & s) ? (((p & ~M0[r]) >> s) | (m & ~M0[r])) : ((m & M0[r]) | ((p & M0[r]) << s));
    }
    return m;
}

__device__ __forceinline__ u32 hslot(i32 w, u32 mask) { return ((u32)w * 2654435761u) & mask; }

// Counting hash (open addressing, linear probing, keys -1 when empty).
// The first slot is probed in straight-line code (it decides almost every
// call at the tables' load); only a slot held by another key sends the lane
// on to the next ones.
__device__ __forceinline__ void hash_add(i32* keys, i32* cnts, u32 mask, i32 w) {
    u32 h = hslot(w, mask);
    i32 old = atomicCAS(&keys[h], -1, w);
    if (old != -1 && old != w) {
        do {
            h = (h + 1) & mask;
            old = atomicCAS(&keys[h], -1, w);
        } while (old != -1 && old != w);
    }
    atomicAdd(&cnts[h], 1);
}

__device__ __forceinline__ i32 hash_get(const i32* keys, const i32* cnts, u32 mask, i32 w) {
    u32 h = hslot(w, mask);
    i32 k = keys[h];
    if (k != w && k != -1) {
        do {
            h = (h + 1) & mask;
            k = keys[h];
        } while (k != w && k != -1);
    }
    return k == w ? cnts[h] : 0;
}

// Position map of up to 2^B distinct vertex ids in 2^B buckets of 4 slots:
// a bucket's keys are one 16-byte LDS word (-1 when empty), so a lookup reads
// one bucket and branches only when the bucket is full and the key is not in
// it (then the next bucket).  Slots of a bucket fill in order, so an empty
// slot ends the search.  Positions are below 2^16.
template <int B>
struct BucketMap {
    int4 key[1 << B];
    u16 pos[4 << B];
};

template <int B>
__device__ __forceinline__ u32 bucket_of(i32 v) {
    return ((u32)v * 2654435761u) >> (32 - B);
}

template <int B>
__device__ __forceinline__ void bmap_clear(BucketMap<B>& m, int tid, int nthreads) {
    for (int q = tid; q < (1 << B); q += nthreads) m.key[q] = make_int4(-1, -1, -1, -1);
}

template <int B>
__device__ __forceinline__ void bmap_insert(BucketMap<B>& m, i32 v, i32 position) {
    u32 b = bucket_of<B>(v);
    i32* keys = reinterpret_cast<i32*>(m.key);
    while (true) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (atomicCAS(&keys[4 * b + s], -1, v) == -1) {
                m.pos[4 * b + s] = (u16)position;
                return;
            }
        }
        b = (b + 1) & ((1u << B) - 1);
    }
}

template <int B>
__device__ __forceinline__ i32 bmap_find(const BucketMap<B>& m, i32 v) {
    // keys are distinct, so at most one slot of a bucket matches; its position
    // is selected directly (one compare and one select per slot), with the
    // bucket's four positions read in the same round trip as its keys.  The
    // first bucket decides almost every lookup; only a full bucket without the
    // key sends the lane on to the next ones.
    u32 b = bucket_of<B>(v);
    int4 q = m.key[b];
    uint2 pp = *reinterpret_cast<const uint2*>(&m.pos[4 * b]);
    auto pick = [&]() {
        i32 r = q.x == v ? (i32)(pp.x & 0xffffu) : -1;
        r = q.y == v ? (i32)(pp.x >> 16) : r;
        r = q.z == v ? (i32)(pp.y & 0xffffu) : r;
        r = q.w == v ? (i32)(pp.y >> 16) : r;
        return r;
    };
    i32 r = pick();
    if (r < 0 && q.w != -1) {
        do {
            b = (b + 1) & ((1u << B) - 1);
            q = m.key[b];
            pp = *reinterpret_cast<const uint2*>(&m.pos[4 * b]);
            r = pick();
        } while (r < 0 && q.w != -1);
    }
    return r;
}

}  // namespace fglt
