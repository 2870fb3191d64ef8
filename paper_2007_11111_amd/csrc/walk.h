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


// Exclusive scan of one value per thread over a block of NT threads; returns
// the thread's prefix and writes the block total to *total.  Every thread of
// the block must call it.
template <int NT, class T>
__device__ __forceinline__ T block_scan(T v, T* wsum, T* total) {
    constexpr int NWV = NT / WAVE;
    const int l = lane_id(), wv = threadIdx.x / WAVE;
    T x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const T y = __shfl_up(x, o, WAVE);
        if (l >= o) x += y;
    }
    if (l == WAVE - 1) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x < WAVE) {
        T y = threadIdx.x < NWV ? wsum[threadIdx.x] : 0;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const T z = __shfl_up(y, o, WAVE);
            if ((int)threadIdx.x >= o) y += z;
        }
        if (threadIdx.x < NWV) wsum[threadIdx.x] = y;
        if (threadIdx.x == NWV - 1) *total = y;
    }
    __syncthreads();
    return (wv > 0 ? wsum[wv - 1] : 0) + x - v;
}

__device__ __forceinline__ i32 block_scan_1024(i32 v, i32* wsum, i32* total) {
    return block_scan<1024>(v, wsum, total);
}

// Walks items [ta, tb) of compacted non-empty runs, 64 consecutive items per
// step.  Run r holds items rstart[r] .. rstart[r+1]-1 at ridx indices
// rbase[r] + item.  The lanes where a run starts are found through a per-wave
// LDS flag row and a ballot.  f(active, item, run, ridx index, run-start mask)
// runs on every lane of the wave.
template <class F>
__device__ __forceinline__ void c4w_walk(i32 ta, i32 tb, const i64* rbase, const i32* rstart, i32 R,
                                         volatile i32* flags, F&& f) {
    if (ta >= tb) return;
    const int l = lane_id();
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    i32 r0 = (i32)last_le_dev(rstart, 0, R - 1, ta);
    for (i32 t0 = ta; t0 < tb; t0 += WAVE) {
        const i32 j = r0 + 1 + l;
        const i32 st = j < R ? rstart[j] : 0x7fffffff;
        // lanes talk through LDS here: volatile accesses in program order, and
        // wavefront barriers so that no store or load moves across the exchange
        flags[l] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (st < t0 + WAVE) flags[st - t0] = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const u64 mask = __ballot(flags[l] != 0);
        __builtin_amdgcn_wave_barrier();
        const i32 r = r0 + __popcll(mask & le);
        const i32 t = t0 + l;
        f(t < tb, t, r, rbase[r] + t, mask);
        r0 = __shfl(r, WAVE - 1, WAVE);
    }
}

// The run walk with U steps in flight: the run masks of U consecutive steps
// are found first, then U independent gathers w = ridx[e] are issued, then
// f(active, item, run, w, e, run-start mask) runs for each step.  Several loads
// per wavefront hide the cache-miss latency that a single load per step exposes.
template <int U, class F>
__device__ __forceinline__ void run_walk(i32 ta, i32 tb, const i64* rbase, const i32* rstart, i32 R,
                                         volatile i32* flags, const i32* __restrict__ ridx, F&& f) {
    if (ta >= tb) return;
    const int l = lane_id();
    const u64 le = l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1);
    i32 r0 = (i32)last_le_dev(rstart, 0, R - 1, ta);
    for (i32 t0 = ta; t0 < tb; t0 += WAVE * U) {
        i32 rr[U];
        u64 mm[U];
        i64 ee[U];
        i32 ww[U];
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 ts = t0 + s * WAVE;
            const i32 j = r0 + 1 + l;
            const i32 st = j < R ? rstart[j] : 0x7fffffff;
            flags[l] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (st < ts + WAVE) flags[st - ts] = 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            mm[s] = __ballot(flags[l] != 0);
            __builtin_amdgcn_wave_barrier();
            rr[s] = r0 + __popcll(mm[s] & le);
            r0 = __shfl(rr[s], WAVE - 1, WAVE);
        }
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 t = t0 + s * WAVE + l;
            ee[s] = t < tb ? rbase[rr[s]] + t : 0;
        }
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 t = t0 + s * WAVE + l;
            ww[s] = t < tb ? ridx[ee[s]] : 0;
        }
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const i32 t = t0 + s * WAVE + l;
            f(t < tb, t, rr[s], ww[s], ee[s], mm[s]);
        }
    }
}

__device__ __forceinline__ u32 hslot(i32 w, u32 mask) { return ((u32)w * 2654435761u) & mask; }

// Counting hash (open addressing, linear probing, keys -1 when empty).
__device__ __forceinline__ void hash_add(i32* keys, i32* cnts, u32 mask, i32 w) {
    u32 h = hslot(w, mask);
    while (true) {
        const i32 old = atomicCAS(&keys[h], -1, w);
        if (old == -1 || old == w) {
            atomicAdd(&cnts[h], 1);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ i32 hash_get(const i32* keys, const i32* cnts, u32 mask, i32 w) {
    u32 h = hslot(w, mask);
    while (true) {
        const i32 k = keys[h];
        if (k == w) return cnts[h];
        if (k == -1) return 0;
        h = (h + 1) & mask;
    }
}

// Position map of a set of distinct vertex ids (insert once, then look up).
__device__ __forceinline__ void pos_insert(i32* keys, i32* vals, u32 mask, i32 v, i32 pos) {
    u32 h = hslot(v, mask);
    while (true) {
        const i32 old = atomicCAS(&keys[h], -1, v);
        if (old == -1) {
            vals[h] = pos;
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ i32 pos_find(const i32* keys, const i32* vals, u32 mask, i32 v) {
    u32 h = hslot(v, mask);
    while (true) {
        const i32 k = keys[h];
        if (k == v) return vals[h];
        if (k == -1) return -1;
        h = (h + 1) & mask;
    }
}

}  // namespace fglt
