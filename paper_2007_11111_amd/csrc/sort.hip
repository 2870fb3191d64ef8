// sort.hip -- segmented ascending sort of non-negative int32 keys, in place.
//
// Segments are classified by length on the device into three work lists:
//   L <= 64        one wavefront per segment: rank by counting (ties by index);
//   64 < L <= 2048 one 256-thread workgroup: bitonic sort in LDS;
//   L > 2048       one 1024-thread workgroup: stable LSD radix sort with 8-bit
//                  digits (wave ballots for in-chunk ranks), ping-ponging
//                  between the segment and the same range of a temp buffer.
// The three sorting kernels walk their list with a grid stride; list lengths
// are read on the device, so no host synchronization is needed.
#include "common.h"

namespace fglt {

static constexpr int SEG_SMALL = 64;
static constexpr int SEG_MID = 2048;
static constexpr int RADIX_THREADS = 1024;

__global__ void k_seg_classify(const i64* __restrict__ seg_off, i64 nseg, i32* __restrict__ lists,
                               i64 list_cap, u32* __restrict__ counters) {
    const i64 s = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    int cls = -1;
    if (s < nseg) {
        const i64 L = seg_off[s + 1] - seg_off[s];
        if (L > 1) cls = L <= SEG_SMALL ? 0 : (L <= SEG_MID ? 1 : 2);
    }
    // wave-aggregated append per class
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const u64 m = __ballot(cls == c);
        if (m == 0) continue;
        const int leader = __ffsll((long long)m) - 1;
        u32 base = 0;
        if (lane_id() == leader) base = atomicAdd(&counters[c], (u32)__popcll(m));
        base = __shfl(base, leader, WAVE);
        if (cls == c) {
            const u32 r = base + (u32)__popcll(m & lanemask_lt());
            lists[(i64)c * list_cap + r] = (i32)s;
        }
    }
}

// One wavefront per segment of length <= 64.
__global__ void __launch_bounds__(256) k_sort_small(i32* __restrict__ keys, const i64* __restrict__ seg_off,
                                                    const i32* __restrict__ list, const u32* __restrict__ count_p) {
    const u32 count = *count_p;
    const i64 wave = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = ((i64)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    for (i64 it = wave; it < (i64)count; it += nwaves) {
        const i64 s = list[it];
        const i64 b = seg_off[s];
        const int L = (int)(seg_off[s + 1] - b);
        const i32 k = l < L ? keys[b + l] : 0x7fffffff;
        int r = 0;
        for (int t = 0; t < L; ++t) {
            const i32 kt = __shfl(k, t, WAVE);
            r += (kt < k) || (kt == k && t < l);
        }
        if (l < L) keys[b + r] = k;
    }
}

// One 256-thread workgroup per segment of length in (64, 2048].
__global__ void __launch_bounds__(256) k_sort_mid(i32* __restrict__ keys, const i64* __restrict__ seg_off,
                                                  const i32* __restrict__ list, const u32* __restrict__ count_p) {
    __shared__ i32 buf[SEG_MID];
    const u32 count = *count_p;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 s = list[it];
        const i64 b = seg_off[s];
        const int L = (int)(seg_off[s + 1] - b);
        int P = 128;
        while (P < L) P <<= 1;
        for (int e = threadIdx.x; e < P; e += blockDim.x) buf[e] = e < L ? keys[b + e] : 0x7fffffff;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int e = threadIdx.x; e < P / 2; e += blockDim.x) {
                    // element pair (i, i ^ j) with i having bit j clear
                    const int i = ((e / j) * 2 * j) + (e % j);
                    const int q = i + j;
                    const bool up = (i & k) == 0;
                    const i32 a = buf[i], c = buf[q];
                    if ((a > c) == up) {
                        buf[i] = c;
                        buf[q] = a;
                    }
                }
                __syncthreads();
            }
        }
        for (int e = threadIdx.x; e < L; e += blockDim.x) keys[b + e] = buf[e];
        __syncthreads();
    }
}

// One 1024-thread workgroup per segment longer than 2048: stable LSD radix.
__global__ void __launch_bounds__(RADIX_THREADS) k_sort_large(i32* __restrict__ keys, i32* __restrict__ tmp,
                                                              const i64* __restrict__ seg_off,
                                                              const i32* __restrict__ list,
                                                              const u32* __restrict__ count_p, int passes) {
    constexpr int NW = RADIX_THREADS / WAVE;
    __shared__ u32 hist[256];
    __shared__ u32 wcnt[NW][256];
    const u32 count = *count_p;
    const int wave = threadIdx.x / WAVE;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 s = list[it];
        const i64 b = seg_off[s];
        const i64 L = seg_off[s + 1] - b;
        i32* src = keys + b;
        i32* dst = tmp + b;
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = 8 * pass;
            for (int e = threadIdx.x; e < 256; e += blockDim.x) hist[e] = 0;
            __syncthreads();
            for (i64 e = threadIdx.x; e < L; e += blockDim.x) atomicAdd(&hist[((u32)src[e] >> shift) & 255u], 1u);
            __syncthreads();
            if (threadIdx.x == 0) {
                u32 run = 0;
                for (int d = 0; d < 256; ++d) {
                    const u32 c = hist[d];
                    hist[d] = run;
                    run += c;
                }
            }
            __syncthreads();
            for (i64 c0 = 0; c0 < L; c0 += RADIX_THREADS) {
                for (int e = threadIdx.x; e < NW * 256; e += blockDim.x) (&wcnt[0][0])[e] = 0;
                __syncthreads();
                const i64 e = c0 + threadIdx.x;
                const bool valid = e < L;
                const i32 k = valid ? src[e] : 0;
                const u32 dgt = ((u32)k >> shift) & 255u;
                u64 m = __ballot(valid);
#pragma unroll
                for (int bit = 0; bit < 8; ++bit) {
                    const u64 bl = __ballot((dgt >> bit) & 1u);
                    m &= ((dgt >> bit) & 1u) ? bl : ~bl;
                }
                const u32 rank_w = (u32)__popcll(m & lanemask_lt());
                if (valid && rank_w == 0) wcnt[wave][dgt] = (u32)__popcll(m);
                __syncthreads();
                if (threadIdx.x < 256) {
                    u32 run = hist[threadIdx.x];
                    for (int w = 0; w < NW; ++w) {
                        const u32 c = wcnt[w][threadIdx.x];
                        wcnt[w][threadIdx.x] = run;
                        run += c;
                    }
                    hist[threadIdx.x] = run;
                }
                __syncthreads();
                if (valid) dst[wcnt[wave][dgt] + rank_w] = k;
                __syncthreads();
            }
            i32* t = src;
            src = dst;
            dst = t;
        }
        if (passes & 1) {
            for (i64 e = threadIdx.x; e < L; e += blockDim.x) keys[b + e] = tmp[b + e];
        }
        __syncthreads();
    }
}

hipError_t seg_sort(i32* keys, const i64* seg_off, i64 nseg, int key_bits, SegSortWs ws, i64 max_seg_grid,
                    hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    hipError_t e = fill_u32(ws.counters, 4, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_classify, dim3((unsigned)ceil_div(nseg, 256)), dim3(256), 0, s, seg_off, nseg,
                       ws.lists, nseg, ws.counters);
    const int passes = key_bits <= 0 ? 1 : (key_bits + 7) / 8;
    const i64 g = max_seg_grid;
    const unsigned g_small = (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(nseg, 4), g));
    const unsigned g_mid = (unsigned)std::max<i64>(1, std::min<i64>(nseg, g));
    const unsigned g_large = (unsigned)std::max<i64>(1, std::min<i64>(nseg, 1024));
    hipLaunchKernelGGL(k_sort_small, dim3(g_small), dim3(256), 0, s, keys, seg_off, ws.lists, ws.counters + 0);
    hipLaunchKernelGGL(k_sort_mid, dim3(g_mid), dim3(256), 0, s, keys, seg_off, ws.lists + nseg, ws.counters + 1);
    hipLaunchKernelGGL(k_sort_large, dim3(g_large), dim3(RADIX_THREADS), 0, s, keys, ws.tmp, seg_off,
                       ws.lists + 2 * nseg, ws.counters + 2, passes);
    return hipGetLastError();
}

}  // namespace fglt
