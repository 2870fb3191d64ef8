// common.h -- internal helpers shared by the HIP sources of libfglt.
// Written for gfx950 (CDNA4): 64-lane wavefronts, 160 KiB LDS per workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fglt.h"

typedef int64_t i64;
typedef int32_t i32;
typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef uint8_t u8;

#define WAVE 64

#define FGLT_HIP_TRY(expr)                          \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return FGLT_EHIP;     \
    } while (0)

#define FGLT_LAUNCH_CHECK()                                   \
    do {                                                      \
        if (hipGetLastError() != hipSuccess) return FGLT_EHIP; \
    } while (0)

// Error bits written by device-side checks into a status word.
enum : u32 {
    ERR_RANGE = 1u,      // an index or offset out of range
    ERR_SELFLOOP = 2u,   // a self-loop
    ERR_DUP = 4u,        // a repeated entry in a row
    ERR_ASYM = 8u,       // an entry (i, j) without (j, i)
    ERR_DEGREE = 16u,    // a degree >= 2^21
};

static inline i64 ceil_div(i64 a, i64 b) { return (a + b - 1) / b; }

// Grid size for `work` items at `per_block` items per workgroup, at least 1, at most cap.
static inline unsigned grid_for(i64 work, i64 per_block, i64 cap = 1 << 20) {
    const i64 g = ceil_div(work > 1 ? work : 1, per_block);
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}
static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Linear allocator over a caller-provided workspace (256-byte aligned pieces;
// up to 255 leading bytes are skipped when the workspace itself is not
// aligned, and the size query reserves them).
struct Carver {
    char* base;
    size_t cap, used;
    explicit Carver(void* b, size_t c) : base((char*)b), cap(c), used(0) {
        used = base ? (size_t)(align_up((size_t)(uintptr_t)base, 256) - (size_t)(uintptr_t)base) : 256;
    }
    template <class T>
    T* take(i64 count) {
        size_t bytes = align_up(sizeof(T) * (size_t)(count > 0 ? count : 1), 256);
        if (base == nullptr) {  // size query
            used += bytes;
            return nullptr;
        }
        if (used + bytes > cap) {
            used += bytes;
            return nullptr;
        }
        T* p = (T*)(base + used);
        used += bytes;
        return p;
    }
    bool ok() const { return base != nullptr && used <= cap; }
};

// Kernels that follow the input checks of fglt_raw take the device error word
// and leave at once when a check has failed, so that a malformed CSR never
// drives an access (the host does not wait for the checks).  Uniform over the
// workgroup; place it before any barrier.
#define FGLT_GATE(errw)                    \
    do {                                   \
        if ((errw) && *(errw)) return;     \
    } while (0)

namespace fglt {
// Fills `words` 32-bit words at p with v, with a kernel (a memset node would be
// recorded into a captured HIP graph).  Defined in scan.hip.
hipError_t fill_u32(void* p, i64 words, u32 v, hipStream_t s);
}  // namespace fglt

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

__device__ __forceinline__ u64 lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ i64 wave_sum(i64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ i64 wave_max(i64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        i64 w = __shfl_xor(v, o, WAVE);
        v = w > v ? w : v;
    }
    return v;
}

// Sum over a workgroup of NT threads, valid on thread 0 (part: NT/64 words of LDS).
template <int NT>
__device__ __forceinline__ i64 block_sum(i64 v, i64* part) {
    v = wave_sum(v);
    if (lane_id() == 0) part[threadIdx.x / WAVE] = v;
    __syncthreads();
    i64 t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / WAVE; ++k) t += part[k];
    __syncthreads();
    return t;
}

template <int NT>
__device__ __forceinline__ i64 block_max(i64 v, i64* part) {
    v = wave_max(v);
    if (lane_id() == 0) part[threadIdx.x / WAVE] = v;
    __syncthreads();
    i64 t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / WAVE; ++k) t = part[k] > t ? part[k] : t;
    __syncthreads();
    return t;
}

// First index q in [lo, hi) with a[q] >= key (hi if none).
template <class T, class K>
__device__ __forceinline__ i64 lower_bound_dev(const T* a, i64 lo, i64 hi, K key) {
    while (lo < hi) {
        i64 mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// lower_bound_dev for an answer expected near hi: probes hi - 1, hi - 2,
// hi - 4, ... (one read when the answer is hi), then a binary search of the
// last gap, so O(log(hi - answer)) reads.
template <class T, class K>
__device__ __forceinline__ i64 lower_bound_back(const T* a, i64 lo, i64 hi, K key) {
    i64 p = hi, step = 1;  // a[p .. hi) >= key
    while (p > lo) {
        const i64 q = p - step > lo ? p - step : lo;
        if (a[q] < key) return lower_bound_dev(a, q + 1, p, key);
        p = q;
        step <<= 1;
    }
    return lo;
}

// lower_bound_dev for an answer expected near lo: probes lo, lo + 1, lo + 3,
// lo + 7, ..., then a binary search of the last gap.
template <class T, class K>
__device__ __forceinline__ i64 lower_bound_fwd(const T* a, i64 lo, i64 hi, K key) {
    i64 p = lo, step = 1;  // a[lo .. p) < key
    while (p < hi) {
        const i64 q = p + step - 1 < hi ? p + step - 1 : hi - 1;
        if (!(a[q] < key)) return lower_bound_dev(a, p, q, key);
        p = q + 1;
        step <<= 1;
    }
    return hi;
}

// Last index r in [lo, hi] with a[r] <= key (lo - 1 if none).
template <class T, class K>
__device__ __forceinline__ i64 last_le_dev(const T* a, i64 lo, i64 hi, K key) {
    i64 l = lo, h = hi + 1;  // search first index with a[idx] > key in [lo, hi+1)
    while (l < h) {
        i64 mid = l + ((h - l) >> 1);
        if (a[mid] <= key) l = mid + 1;
        else h = mid;
    }
    return l - 1;
}

// Row r of a CSR entry p: roff[r] <= p < roff[r+1], searched in [rlo, rhi].
__device__ __forceinline__ i64 row_of(const i64* roff, i64 rlo, i64 rhi, i64 p) {
    return last_le_dev(roff, rlo, rhi, p);
}

// Inclusive segmented sum across a wave: lanes with equal `key` that are
// contiguous form one segment; returns the running sum within the segment.
__device__ __forceinline__ i64 wave_seg_scan(i64 v, i64 key) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        i64 u = __shfl_up(v, o, WAVE);
        i64 k = __shfl_up(key, o, WAVE);
        if (l >= o && k == key) v += u;
    }
    return v;
}

// True on the last lane of each contiguous run of equal keys.
__device__ __forceinline__ bool wave_seg_tail(i64 key, bool active) {
    const int l = lane_id();
    i64 next = __shfl_down(key, 1, WAVE);
    int next_active = __shfl_down((int)active, 1, WAVE);
    return active && (l == WAVE - 1 || !next_active || next != key);
}

// One atomic per run of equal keys instead of one per lane: for lanes whose
// keys are non-decreasing across the wavefront and whose active lanes form a
// prefix of it, the first lane of each run adds the number of the run's lanes
// with `hit` set to a[key].  Call with every active lane.
template <class T>
__device__ __forceinline__ void wave_run_add(T* a, i64 key, bool hit) {
    const int l = lane_id();
    const u64 hm = __ballot(hit);
    const i64 prev = __shfl_up(key, 1, WAVE);
    const bool head = l == 0 || prev != key;
    const u64 hd = __ballot(head);
    if (head) {
        const u64 later = l == WAVE - 1 ? 0ull : hd & (~0ull << (l + 1));  // heads after this lane
        const u64 upto = later ? (later & (0ull - later)) - 1ull : ~0ull;  // lanes below the next head
        const int c = __popcll(hm & upto & (~0ull << l));
        if (c) atomicAdd(&a[key], (T)c);
    }
}

// ---------------------------------------------------------------- host launch helpers

namespace fglt {

hipError_t scan_exclusive_i64(const i64* in, i64* out, i64 count, i64* partials, hipStream_t s);
hipError_t scan_exclusive_i32_to_i64(const i32* in, i64* out, i64 count, i64* partials, hipStream_t s);
i64 scan_partials_size(i64 count);

struct SegSortWs {
    i32* tmp;       // [max total keys]
    i32* lists;     // [3 * max segments]
    u32* counters;  // [4]
};
hipError_t seg_sort(i32* keys, const i64* seg_off, i64 nseg, int key_bits, SegSortWs ws,
                    i64 max_seg_grid, hipStream_t s);

// Stable LSD radix sort of n pairs (in_k, in_v) by the low key_bits bits of
// the keys (keys below 2^key_bits) into (out_k, out_v).  in_v == nullptr means
// values 0 .. n-1; out_k == nullptr skips the sorted keys.  Passes alternate
// through (ta_k, ta_v) and (tb_k, tb_v), n words each; tb may be the memory
// of in_k / in_v (read only by the first pass), ta may not.  hist holds
// radix_hist_size(n) words; partials as for scan_exclusive_i64 of that many.
i64 radix_hist_size(i64 n);
hipError_t radix_sort_pairs(i64 n, int key_bits, const u32* in_k, const i32* in_v, u32* out_k, i32* out_v,
                            u32* ta_k, i32* ta_v, u32* tb_k, i32* tb_v, i64* hist, i64* partials, hipStream_t s);

}  // namespace fglt
