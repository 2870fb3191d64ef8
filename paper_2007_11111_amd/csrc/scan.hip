// scan.hip -- device-wide exclusive prefix sums (int32/int64 in, int64 out).
//
// Three launches: per-tile sums, one-workgroup scan of the tile sums, per-tile
// scan with the tile's prefix added.  out has count+1 entries; out[count] is
// the total.  out may alias in (each tile is read completely before it is
// written, and tiles are disjoint).
#include "common.h"

namespace fglt {

static constexpr int SCAN_THREADS = 256;
static constexpr int SCAN_ITEMS = 8;
static constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

i64 scan_partials_size(i64 count) { return ceil_div(count > 0 ? count : 1, SCAN_TILE) + 1; }

template <class T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const T* __restrict__ in, i64 count,
                                                            i64* __restrict__ partials) {
    __shared__ i64 red[SCAN_THREADS / WAVE];
    const i64 base = (i64)blockIdx.x * SCAN_TILE;
    i64 s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        i64 p = base + (i64)k * SCAN_THREADS + threadIdx.x;
        if (p < count) s += (i64)in[p];
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        i64 t = 0;
        for (int w = 0; w < SCAN_THREADS / WAVE; ++w) t += red[w];
        partials[blockIdx.x] = t;
    }
}

// Exclusive scan of partials[0..nb) in place, with partials[nb] = total.
__global__ void __launch_bounds__(1024) k_scan_partials(i64* __restrict__ partials, i64 nb) {
    __shared__ i64 wsum[1024 / WAVE];
    __shared__ i64 carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (i64 base = 0; base < nb; base += 1024) {
        const i64 p = base + threadIdx.x;
        const i64 v = p < nb ? partials[p] : 0;
        // inclusive wave scan
        i64 x = v;
        const int l = lane_id();
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            i64 u = __shfl_up(x, o, WAVE);
            if (l >= o) x += u;
        }
        if (l == WAVE - 1) wsum[threadIdx.x / WAVE] = x;
        __syncthreads();
        if (threadIdx.x < WAVE) {
            i64 y = threadIdx.x < 1024 / WAVE ? wsum[threadIdx.x] : 0;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                i64 u = __shfl_up(y, o, WAVE);
                if ((int)threadIdx.x >= o) y += u;
            }
            if (threadIdx.x < 1024 / WAVE) wsum[threadIdx.x] = y;  // inclusive over waves
        }
        __syncthreads();
        const int w = threadIdx.x / WAVE;
        const i64 carry = carry_s;
        const i64 excl = carry + (w > 0 ? wsum[w - 1] : 0) + x - v;
        if (p < nb) partials[p] = excl;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + wsum[1024 / WAVE - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[nb] = carry_s;
}

template <class T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_scan(const T* __restrict__ in, i64* __restrict__ out,
                                                            i64 count, const i64* __restrict__ partials) {
    __shared__ i64 tile[SCAN_TILE];
    __shared__ i64 wsum[SCAN_THREADS / WAVE];
    const i64 base = (i64)blockIdx.x * SCAN_TILE;
    // coalesced load into LDS
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int e = k * SCAN_THREADS + threadIdx.x;
        const i64 p = base + e;
        tile[e] = p < count ? (i64)in[p] : 0;
    }
    __syncthreads();
    // thread t owns tile[t*ITEMS .. t*ITEMS + ITEMS)
    i64 v[SCAN_ITEMS];
    i64 tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = tile[threadIdx.x * SCAN_ITEMS + k];
        tsum += v[k];
    }
    i64 x = tsum;
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        i64 u = __shfl_up(x, o, WAVE);
        if (l >= o) x += u;
    }
    if (l == WAVE - 1) wsum[threadIdx.x / WAVE] = x;
    __syncthreads();
    const int w = threadIdx.x / WAVE;
    i64 pre = partials[blockIdx.x] + x - tsum;
    for (int q = 0; q < w; ++q) pre += wsum[q];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        tile[threadIdx.x * SCAN_ITEMS + k] = pre;
        pre += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int e = k * SCAN_THREADS + threadIdx.x;
        const i64 p = base + e;
        if (p < count) out[p] = tile[e];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = partials[gridDim.x];
}

__global__ void k_fill_u32(u32* __restrict__ p, i64 words, u32 v) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t fill_u32(void* p, i64 words, u32 v, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, 256, 16384)), dim3(256), 0, s, (u32*)p, words, v);
    return hipGetLastError();
}

template <class T>
static hipError_t scan_impl(const T* in, i64* out, i64 count, i64* partials, hipStream_t s) {
    if (count <= 0) return fill_u32(out, 2, 0u, s);
    const i64 nb = ceil_div(count, SCAN_TILE);
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, count, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, nb);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, out, count, partials);
    return hipGetLastError();
}

hipError_t scan_exclusive_i64(const i64* in, i64* out, i64 count, i64* partials, hipStream_t s) {
    return scan_impl<i64>(in, out, count, partials, s);
}

hipError_t scan_exclusive_i32_to_i64(const i32* in, i64* out, i64 count, i64* partials, hipStream_t s) {
    return scan_impl<i32>(in, out, count, partials, s);
}

}  // namespace fglt
