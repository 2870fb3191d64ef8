// radix.hip -- stable LSD radix sort of (key, value) pairs, 8-bit digits.
//
// One pass per digit, three launches each:
//   count:   per tile of RX_TILE consecutive pairs, the count of each digit,
//            stored digit-major (cnt[d * ntiles + tile]);
//   scan:    exclusive scan of that array, giving each (digit, tile) its
//            first output position (all smaller digits, then earlier tiles);
//   scatter: each tile ranks its pairs stably -- a wavefront takes 64 * RX_ITEMS
//            consecutive pairs in RX_ITEMS steps of 64; lanes with equal
//            digits find each other with 8 ballots, and a per-wavefront LDS
//            counter per digit carries the ranks from step to step -- then
//            places them in LDS in digit order and writes each digit's pairs
//            as one run of consecutive lanes.
// Stable passes from the least significant digit up leave the pairs ordered
// by key, ties in input order.
#include "walk.h"

namespace fglt {

static constexpr int RX_BITS = 8;
static constexpr int RX_DIG = 1 << RX_BITS;
static constexpr int RX_THREADS = 256;  // one thread per digit in the per-digit loops
static constexpr int RX_NW = RX_THREADS / WAVE;
static constexpr int RX_ITEMS = 16;
static constexpr i64 RX_TILE = (i64)RX_THREADS * RX_ITEMS;
static_assert(RX_THREADS == RX_DIG, "the per-digit loops use one thread per digit");

i64 radix_hist_size(i64 n) { return RX_DIG * std::max<i64>(1, ceil_div(n, RX_TILE)); }

__global__ void __launch_bounds__(RX_THREADS) k_rx_count(const u32* __restrict__ keys, i64 n, int shift,
                                                         i64 ntiles, i64* __restrict__ cnt) {
    __shared__ u32 h[RX_DIG];
    for (i64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        h[threadIdx.x] = 0;
        __syncthreads();
        const i64 t0 = tile * RX_TILE;
#pragma unroll
        for (int j = 0; j < RX_ITEMS; ++j) {
            const i64 i = t0 + (i64)j * RX_THREADS + threadIdx.x;
            if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RX_DIG - 1)], 1u);
        }
        __syncthreads();
        cnt[(i64)threadIdx.x * ntiles + tile] = h[threadIdx.x];
        __syncthreads();
    }
}

// vals == nullptr: the value of pair i is i.  out_k == nullptr: keys not written.
// The ranked tile is staged in LDS in digit order, so that the pairs of one
// digit leave as one contiguous run of consecutive lanes.
__global__ void __launch_bounds__(RX_THREADS) k_rx_scatter(const u32* __restrict__ keys, const i32* __restrict__ vals,
                                                           i64 n, int shift, i64 ntiles, const i64* __restrict__ off,
                                                           u32* __restrict__ out_k, i32* __restrict__ out_v) {
    __shared__ i32 wc[RX_NW][RX_DIG];  // per wavefront: pairs of each digit so far, then its first tile slot
    __shared__ i64 gofs[RX_DIG];       // output position of digit d minus its first tile slot
    __shared__ u32 sk[RX_TILE];
    __shared__ i32 sv[RX_TILE];
    __shared__ i32 wsum[RX_NW], wtot;
    const int wv = threadIdx.x / WAVE, l = lane_id();
    const u64 lt = lanemask_lt();
    for (i64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        for (int w = 0; w < RX_NW; ++w) wc[w][threadIdx.x] = 0;
        __syncthreads();
        const i64 t0 = tile * RX_TILE;
        const i64 w0 = t0 + (i64)wv * WAVE * RX_ITEMS;
        u32 kk[RX_ITEMS];
        i32 vv[RX_ITEMS];
#pragma unroll
        for (int j = 0; j < RX_ITEMS; ++j) {
            const i64 i = w0 + (i64)j * WAVE + l;
            kk[j] = i < n ? keys[i] : 0u;
            vv[j] = i < n ? (vals ? vals[i] : (i32)i) : 0;
        }
        i32 rk[RX_ITEMS];
#pragma unroll
        for (int j = 0; j < RX_ITEMS; ++j) {
            const bool valid = w0 + (i64)j * WAVE + l < n;
            const u32 d = (kk[j] >> shift) & (RX_DIG - 1);
            u64 m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < RX_BITS; ++b) {
                const bool bit = (d >> b) & 1u;
                const u64 bl = __ballot(bit);
                m &= bit ? bl : ~bl;
            }
            // m: the valid lanes with this lane's digit
            const i32 prior = valid ? lds_get(&wc[wv][d]) : 0;
            rk[j] = prior + __popcll(m & lt);
            wave_lds_fence();
            if (valid && (m & lt) == 0) lds_put(&wc[wv][d], prior + __popcll(m));
            wave_lds_fence();
        }
        __syncthreads();
        {
            // digit d: its tile slots start after all smaller digits; within
            // the digit, wavefront w's pairs follow those of wavefronts < w
            const int d = threadIdx.x;
            i32 c[RX_NW], tot = 0;
#pragma unroll
            for (int w = 0; w < RX_NW; ++w) {
                c[w] = wc[w][d];
                tot += c[w];
            }
            const i32 start = block_scan<RX_THREADS>(tot, wsum, &wtot);
            i32 run = start;
#pragma unroll
            for (int w = 0; w < RX_NW; ++w) {
                wc[w][d] = run;
                run += c[w];
            }
            gofs[d] = off[(i64)d * ntiles + tile] - start;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RX_ITEMS; ++j) {
            if (w0 + (i64)j * WAVE + l < n) {
                const i32 slot = wc[wv][(kk[j] >> shift) & (RX_DIG - 1)] + rk[j];
                sk[slot] = kk[j];
                sv[slot] = vv[j];
            }
        }
        __syncthreads();
        const i32 cnt = (i32)std::min<i64>(RX_TILE, n - t0);
        for (i32 i = threadIdx.x; i < cnt; i += RX_THREADS) {
            const u32 k = sk[i];
            const i64 pos = gofs[(k >> shift) & (RX_DIG - 1)] + i;
            out_v[pos] = sv[i];
            if (out_k) out_k[pos] = k;
        }
        __syncthreads();
    }
}

hipError_t radix_sort_pairs(i64 n, int key_bits, const u32* in_k, const i32* in_v, u32* out_k, i32* out_v,
                            u32* ta_k, i32* ta_v, u32* tb_k, i32* tb_v, i64* hist, i64* partials, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int passes = std::max(1, (key_bits + RX_BITS - 1) / RX_BITS);
    const i64 ntiles = ceil_div(n, RX_TILE);
    const unsigned grid = (unsigned)std::min<i64>(ntiles, 65536);
    const u32* sk = in_k;
    const i32* sv = in_v;
    for (int p = 0; p < passes; ++p) {
        const bool last = p == passes - 1;
        u32* dk = last ? out_k : (p % 2 == 0 ? ta_k : tb_k);
        i32* dv = last ? out_v : (p % 2 == 0 ? ta_v : tb_v);
        const int shift = RX_BITS * p;
        hipLaunchKernelGGL(k_rx_count, dim3(grid), dim3(RX_THREADS), 0, s, sk, n, shift, ntiles, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if ((e = scan_exclusive_i64(hist, hist, RX_DIG * ntiles, partials, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_rx_scatter, dim3(grid), dim3(RX_THREADS), 0, s, sk, sv, n, shift, ntiles, hist, dk, dv);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        sk = dk;
        sv = dv;
    }
    return hipSuccess;
}

}  // namespace fglt
