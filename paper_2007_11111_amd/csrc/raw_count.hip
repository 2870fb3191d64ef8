// raw_count.hip -- the counting passes of the transform, in rank space.
//
//   L1  row pass:   sum_j d_j (-> p2 = A p1 - p1) and sum_j C(d_j - 1, 2) (-> \hat d_7)
//   TRI mode 1:     oriented triangle listing per vertex u over N+(u); C3 on
//                   every oriented edge and c3 per vertex (C3 = A .* A^2, Lemma 2)
//   FILL:           C3 copied to the mirrored entries
//   L2  row pass:   A p2, A c3, C3 (p1 - 2), sum_j C(C3(i,j), 2)   (Table I rows 5, 9, 10, 14)
//   TRI mode 2:     the induced subgraph on N+(u) as LDS bitmaps; per vertex
//                   4-cliques (T e / 6, Section IV-C) and off-cord diamonds
//                   (D4,c e / 2) attributed to all four / three vertices
//   C4:             rank-ordered wedges u - v - w with v, w < u, counted in an
//                   LDS hash (or a dense global array for heavy u); 4-cycles
//                   (C4,2 e / 2, Lemma 5) attributed to u, w and the middles
//   FINALIZE:       Table I assembled per vertex, Table II back-substitution,
//                   rows scattered back to the caller's vertex order
#include <algorithm>

#include "walk.h"

namespace fglt {

static constexpr int PT = 256;

static inline unsigned grid_for(i64 work, i64 per_block, i64 cap = 1 << 20) {
    return (unsigned)std::max<i64>(1, std::min<i64>(ceil_div(std::max<i64>(work, 1), per_block), cap));
}

static int bits_for_n(i64 n) {
    int b = 0;
    while (b < 31 && (((i64)1 << b) <= n - 1)) ++b;
    return b;
}

__device__ __forceinline__ void fence_agent() { __threadfence(); }

__device__ __forceinline__ i32 load_relaxed(const i32* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ row passes

__global__ void __launch_bounds__(PT) k_l1(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                           const i32* __restrict__ rdeg, i64 n, i64 nnz, i64* __restrict__ sumd,
                                           i64* __restrict__ s7) {
    const i64 nw = ((i64)gridDim.x * blockDim.x) / WAVE;
    for (i64 wv = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; wv * WAVE < nnz; wv += nw) {
        const i64 p0 = wv * WAVE;
        const i64 pl = std::min<i64>(p0 + WAVE - 1, nnz - 1);
        const i64 r0 = row_of(roff, 0, n - 1, p0);
        const i64 r1 = row_of(roff, r0, n - 1, pl);
        const i64 p = p0 + lane_id();
        const bool act = p < nnz;
        i64 r = -1, a = 0, b = 0;
        if (act) {
            r = row_of(roff, r0, r1, p);
            const i64 dj = rdeg[ridx[p]];
            a = dj;
            b = (dj - 1) * (dj - 2) / 2;
        }
        a = wave_seg_scan(a, r);
        b = wave_seg_scan(b, r);
        if (wave_seg_tail(r, act)) {
            atomicAdd((unsigned long long*)&sumd[r], (unsigned long long)a);
            if (b) atomicAdd((unsigned long long*)&s7[r], (unsigned long long)b);
        }
    }
}

__global__ void __launch_bounds__(PT) k_l2(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                           const i32* __restrict__ rdeg, const i32* __restrict__ C3,
                                           const i64* __restrict__ sumd, const i64* __restrict__ c3v, i64 n,
                                           i64 nnz, i64* __restrict__ ap2, i64* __restrict__ ac3,
                                           i64* __restrict__ d10, i64* __restrict__ d14) {
    const i64 nw = ((i64)gridDim.x * blockDim.x) / WAVE;
    for (i64 wv = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; wv * WAVE < nnz; wv += nw) {
        const i64 p0 = wv * WAVE;
        const i64 pl = std::min<i64>(p0 + WAVE - 1, nnz - 1);
        const i64 r0 = row_of(roff, 0, n - 1, p0);
        const i64 r1 = row_of(roff, r0, n - 1, pl);
        const i64 p = p0 + lane_id();
        const bool act = p < nnz;
        i64 r = -1, a = 0, b = 0, c = 0, d = 0;
        if (act) {
            r = row_of(roff, r0, r1, p);
            const i32 j = ridx[p];
            const i64 dj = rdeg[j];
            const i64 t = C3[p];
            a = sumd[j] - dj;          // p2(j)
            b = c3v[j];                // c3(j)
            c = t * (dj - 2);          // C3(i,j) (p1(j) - 2); t == 0 when dj == 1
            d = t * (t - 1) / 2;       // C(C3(i,j), 2)
        }
        a = wave_seg_scan(a, r);
        b = wave_seg_scan(b, r);
        c = wave_seg_scan(c, r);
        d = wave_seg_scan(d, r);
        if (wave_seg_tail(r, act)) {
            if (a) atomicAdd((unsigned long long*)&ap2[r], (unsigned long long)a);
            if (b) atomicAdd((unsigned long long*)&ac3[r], (unsigned long long)b);
            if (c) atomicAdd((unsigned long long*)&d10[r], (unsigned long long)c);
            if (d) atomicAdd((unsigned long long*)&d14[r], (unsigned long long)d);
        }
    }
}

__global__ void k_fill_c3(const i64* __restrict__ roff, const i32* __restrict__ ridx, const i32* __restrict__ rpos,
                          i64 nnz, i32* __restrict__ C3) {
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (i64)gridDim.x * blockDim.x) {
        const i32 rp = rpos[p];
        if (rp >= 0) C3[p] = C3[roff[ridx[p]] + rp];
    }
}

// ------------------------------------------------------------ triangle / clique passes


// Wave tier: out-degree D in [2, 64]; one wavefront per vertex, 4 per block.
template <int MODE>
__global__ void __launch_bounds__(PT) k_tri_wave(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                 const i32* __restrict__ lo, const i32* __restrict__ rdeg,
                                                 const i64* __restrict__ G, const i32* __restrict__ list, u32 count,
                                                 i32* __restrict__ C3, i64* __restrict__ c3v, i64* __restrict__ k4v,
                                                 i64* __restrict__ d13, DevPlan* plan) {
    constexpr int NW = PT / WAVE;
    __shared__ i32 sL[NW][WAVE];
    __shared__ i32 sPre[NW][WAVE + 1];
    __shared__ i64 sBv[NW][WAVE];
    __shared__ i32 sCnt[NW][WAVE];
    __shared__ u64 sB[NW][MODE == 2 ? WAVE : 1];
    __shared__ u64 sC[NW][MODE == 2 ? WAVE : 1];
    const int wid = threadIdx.x / WAVE;
    const int lane = lane_id();
    for (i64 base = (i64)blockIdx.x * NW; base < (i64)count; base += (i64)gridDim.x * NW) {
        const i64 it = base + wid;
        const bool valid = it < (i64)count;
        i64 u = 0, bu = 0, gb = 0;
        int D = 0, T = 0;
        if (valid) {
            u = list[it];
            bu = roff[u] + lo[u];
            D = (int)(roff[u + 1] - bu);
            gb = G[bu];
            T = (int)(G[bu + D] - gb);
            if (lane < D) {
                const i32 v = ridx[bu + lane];
                sL[wid][lane] = v;
                sBv[wid][lane] = roff[v] + lo[v];
                sPre[wid][lane] = (i32)(G[bu + lane] - gb);
                if (MODE == 1) {
                    sCnt[wid][lane] = 0;
                } else {
                    sCnt[wid][lane] = C3[bu + lane];
                    sB[wid][lane] = 0;
                    sC[wid][lane] = 0;
                }
            }
            if (lane == 0) sPre[wid][D] = T;
        }
        __syncthreads();
        i64 d13u = 0;
        for (int t = lane; t < T; t += WAVE) {
            const int k = (int)last_le_dev(sPre[wid], 0, D - 1, t);
            const int o = t - sPre[wid][k];
            const i64 e = sBv[wid][k] + o;
            const i32 y = ridx[e];
            const int l = (int)lower_bound_dev(sL[wid], (i64)k + 1, (i64)D, y);
            if (l < D && sL[wid][l] == y) {
                if (MODE == 1) {
                    atomicAdd(&sCnt[wid][k], 1);
                    atomicAdd(&sCnt[wid][l], 1);
                    atomicAdd(&C3[e], 1);
                } else {
                    atomicOr((unsigned long long*)&sB[wid][k], 1ull << l);
                    atomicOr((unsigned long long*)&sC[wid][l], 1ull << k);
                    d13u += (i64)C3[e] - 1;
                }
            }
        }
        __syncthreads();
        if (valid) {
            if (MODE == 1) {
                i64 c = 0;
                if (lane < D) {
                    c = sCnt[wid][lane];
                    if (c) {
                        atomicAdd(&C3[bu + lane], (i32)c);
                        atomicAdd((unsigned long long*)&c3v[sL[wid][lane]], (unsigned long long)c);
                    }
                }
                c = wave_sum(c);
                if (lane == 0 && c) {
                    atomicAdd((unsigned long long*)&c3v[u], (unsigned long long)(c / 2));
                    atomicAdd((unsigned long long*)&plan->triangles, (unsigned long long)(c / 2));
                }
            } else {
                i64 R = 0, kv = 0, dv = 0;
                if (lane < D) {
                    const u64 Bk = sB[wid][lane], Ck = sC[wid][lane];
                    FOR_BITS(Bk, l, {
                        R += __popcll(Bk & sB[wid][l]);
                        dv += sCnt[wid][l] - 1;
                    });
                    i64 M = 0, X = 0;
                    FOR_BITS(Ck, j, {
                        const u64 Bj = sB[wid][j];
                        M += __popcll(Bj & Bk);
                        X += __popcll(Bj & Ck);
                        dv += sCnt[wid][j] - 1;
                    });
                    kv = R + M + X;
                    if (kv) atomicAdd((unsigned long long*)&k4v[sL[wid][lane]], (unsigned long long)kv);
                    if (dv) atomicAdd((unsigned long long*)&d13[sL[wid][lane]], (unsigned long long)dv);
                }
                R = wave_sum(R);
                d13u = wave_sum(d13u);
                if (lane == 0) {
                    if (R) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)R);
                    if (d13u) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)d13u);
                }
            }
        } else {
            d13u = wave_sum(d13u);  // keep the wave's collectives uniform
        }
        __syncthreads();
    }
}

// Workgroup tiers: out-degree D > 64.  GLOBAL = false keeps bitmaps and lists
// in LDS (D <= TRI_LDS_MAX); GLOBAL = true keeps them in a per-block slot of
// device memory (any D up to sqrt(nnz)).
template <int MODE, bool GLOBAL>
__global__ void __launch_bounds__(PT) k_tri_block(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                  const i32* __restrict__ lo, const i32* __restrict__ rdeg,
                                                  const i64* __restrict__ G, const i32* __restrict__ list,
                                                  u32 count, i32* __restrict__ C3, i64* __restrict__ c3v,
                                                  i64* __restrict__ k4v, i64* __restrict__ d13,
                                                  u64* __restrict__ slots, i64 slot_words, DevPlan* plan) {
    constexpr int DM = TRI_LDS_MAX;
    constexpr int WM = DM / 64;
    constexpr bool BITS = MODE == 2;
    __shared__ i32 lL[GLOBAL ? 1 : DM];
    __shared__ i32 lPre[GLOBAL ? 1 : DM + 1];
    __shared__ i64 lBv[GLOBAL ? 1 : DM];
    __shared__ i32 lCnt[GLOBAL ? 1 : DM];
    __shared__ u64 lB[(GLOBAL || !BITS) ? 1 : DM * WM];
    __shared__ u64 lC[(GLOBAL || !BITS) ? 1 : DM * WM];
    __shared__ i64 red[2];

    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        const int W = (D + 63) / 64;
        const i64 gb = G[bu];
        const i64 T = G[bu + D] - gb;
        i32 *L, *Pre, *Cnt;
        i64* Bv;
        u64 *B, *C;
        if (GLOBAL) {
            u64* sl = slots + (i64)blockIdx.x * slot_words;
            B = sl;
            C = sl + (i64)D * W;
            u64* rest = C + (i64)D * W;
            Bv = (i64*)rest;
            L = (i32*)(rest + D);
            Pre = L + D;               // D + 1 entries
            Cnt = Pre + D + 2;         // D entries
        } else {
            L = lL;
            Pre = lPre;
            Bv = lBv;
            Cnt = lCnt;
            B = lB;
            C = lC;
        }
        // Pre holds offsets relative to gb; T may exceed 2^31 only for D beyond the LDS tier,
        // where Pre is read from G directly instead.
        for (int k = threadIdx.x; k < D; k += blockDim.x) {
            const i32 v = ridx[bu + k];
            L[k] = v;
            Bv[k] = roff[v] + lo[v];
            if (!GLOBAL) Pre[k] = (i32)(G[bu + k] - gb);
            Cnt[k] = MODE == 1 ? 0 : C3[bu + k];
        }
        if (BITS) {
            for (i64 q = threadIdx.x; q < (i64)D * W; q += blockDim.x) {
                B[q] = 0;
                C[q] = 0;
            }
        }
        if (threadIdx.x == 0) {
            if (!GLOBAL) Pre[D] = (i32)T;
            red[0] = 0;
            red[1] = 0;
        }
        if (GLOBAL) fence_agent();
        __syncthreads();
        if (GLOBAL) fence_agent();

        i64 d13u = 0;
        for (i64 t = threadIdx.x; t < T; t += blockDim.x) {
            int k;
            i64 o;
            if (GLOBAL) {
                const i64 q = last_le_dev(G, bu, bu + D - 1, gb + t);
                k = (int)(q - bu);
                o = gb + t - G[q];
            } else {
                k = (int)last_le_dev(Pre, 0, D - 1, (i32)t);
                o = t - Pre[k];
            }
            const i64 e = Bv[k] + o;
            const i32 y = ridx[e];
            const int l = (int)lower_bound_dev(L, (i64)k + 1, (i64)D, y);
            if (l < D && L[l] == y) {
                if (MODE == 1) {
                    atomicAdd(&Cnt[k], 1);
                    atomicAdd(&Cnt[l], 1);
                    atomicAdd(&C3[e], 1);
                } else {
                    atomicOr((unsigned long long*)&B[(i64)k * W + (l >> 6)], 1ull << (l & 63));
                    atomicOr((unsigned long long*)&C[(i64)l * W + (k >> 6)], 1ull << (k & 63));
                    d13u += (i64)C3[e] - 1;
                }
            }
        }
        if (GLOBAL) fence_agent();
        __syncthreads();
        if (GLOBAL) fence_agent();

        if (MODE == 1) {
            i64 c = 0;
            for (int k = threadIdx.x; k < D; k += blockDim.x) {
                const i64 ck = GLOBAL ? (i64)load_relaxed(&Cnt[k]) : (i64)Cnt[k];
                if (ck) {
                    atomicAdd(&C3[bu + k], (i32)ck);
                    atomicAdd((unsigned long long*)&c3v[L[k]], (unsigned long long)ck);
                }
                c += ck;
            }
            c = wave_sum(c);
            if (lane_id() == 0 && c) atomicAdd((unsigned long long*)&red[0], (unsigned long long)c);
        } else {
            i64 Rsum = 0;
            for (int k = threadIdx.x; k < D; k += blockDim.x) {
                const u64* Bk = B + (i64)k * W;
                const u64* Ck = C + (i64)k * W;
                i64 R = 0, M = 0, X = 0, dv = 0;
                for (int wa = 0; wa < W; ++wa) {
                    FOR_BITS(Bk[wa], bb, {
                        const int l = wa * 64 + bb;
                        const u64* Bl = B + (i64)l * W;
                        for (int z = 0; z < W; ++z) R += __popcll(Bk[z] & Bl[z]);
                        dv += Cnt[l] - 1;
                    });
                    FOR_BITS(Ck[wa], bb, {
                        const int j = wa * 64 + bb;
                        const u64* Bj = B + (i64)j * W;
                        for (int z = 0; z < W; ++z) {
                            M += __popcll(Bj[z] & Bk[z]);
                            X += __popcll(Bj[z] & Ck[z]);
                        }
                        dv += Cnt[j] - 1;
                    });
                }
                const i64 kv = R + M + X;
                if (kv) atomicAdd((unsigned long long*)&k4v[L[k]], (unsigned long long)kv);
                if (dv) atomicAdd((unsigned long long*)&d13[L[k]], (unsigned long long)dv);
                Rsum += R;
            }
            Rsum = wave_sum(Rsum);
            d13u = wave_sum(d13u);
            if (lane_id() == 0) {
                if (Rsum) atomicAdd((unsigned long long*)&red[0], (unsigned long long)Rsum);
                if (d13u) atomicAdd((unsigned long long*)&red[1], (unsigned long long)d13u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (MODE == 1) {
                if (red[0]) {
                    atomicAdd((unsigned long long*)&c3v[u], (unsigned long long)(red[0] / 2));
                    atomicAdd((unsigned long long*)&plan->triangles, (unsigned long long)(red[0] / 2));
                }
            } else {
                if (red[0]) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)red[0]);
                if (red[1]) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)red[1]);
            }
        }
        if (GLOBAL) fence_agent();
        __syncthreads();
    }
}

// ------------------------------------------------------------ 4-cycle pass

// Wedge item t of vertex u (N- entries in [b, m)): the entry q = (u, v) and the
// wedge end w = the o-th neighbour of v.
__device__ __forceinline__ void wedge_item(const i64* __restrict__ G, const i64* __restrict__ roff,
                                           const i32* __restrict__ ridx, i64 b, i64 m, i64 g, i64& q, i32& w) {
    q = last_le_dev(G, b, m - 1, g);
    const i32 v = ridx[q];
    w = ridx[roff[v] + (g - G[q])];
}

// LDS-hash tiers.  WAVES_PER_U = 1: one wavefront per vertex (4 per block,
// 256-slot table each); WAVES_PER_U = 4: the whole block on one vertex with a
// 4096-slot table.
template <int WAVES_PER_U, int HSLOTS>
__global__ void __launch_bounds__(PT) k_c4_hash(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                const i32* __restrict__ lo, const i64* __restrict__ G,
                                                const i32* __restrict__ list, u32 count, i64* __restrict__ c4v) {
    constexpr int NW = PT / WAVE;
    constexpr int GROUPS = NW / WAVES_PER_U;  // vertices per block
    constexpr int GT = WAVES_PER_U * WAVE;    // threads per vertex
    __shared__ i32 hk[GROUPS][HSLOTS];
    __shared__ i32 hc[GROUPS][HSLOTS];
    __shared__ i64 red[GROUPS];
    const int grp = threadIdx.x / GT;
    const int gt = threadIdx.x % GT;
    const u32 mask = HSLOTS - 1;
    for (i64 base = (i64)blockIdx.x * GROUPS; base < (i64)count; base += (i64)gridDim.x * GROUPS) {
        const i64 it = base + grp;
        const bool valid = it < (i64)count;
        i64 u = 0, b = 0, m = 0, gb = 0, W = 0;
        if (valid) {
            u = list[it];
            b = roff[u];
            m = b + lo[u];
            gb = G[b];
            W = G[m] - gb;
        }
        for (int s = gt; s < HSLOTS; s += GT) {
            hk[grp][s] = -1;
            hc[grp][s] = 0;
        }
        if (gt == 0) red[grp] = 0;
        __syncthreads();
        // pass A: count wedge ends
        for (i64 t = gt; t < W; t += GT) {
            i64 q;
            i32 w;
            wedge_item(G, roff, ridx, b, m, gb + t, q, w);
            hash_add(hk[grp], hc[grp], mask, w);
        }
        __syncthreads();
        // pass B: C(cnt, 2) to u and to w
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
        // pass C: cnt(w) - 1 to the middle vertex of every wedge
        for (i64 t0 = 0; t0 < W; t0 += GT) {
            const i64 t = t0 + gt;
            const bool act = t < W;
            i64 q = -1, val = 0;
            if (act) {
                i32 w;
                wedge_item(G, roff, ridx, b, m, gb + t, q, w);
                val = hash_get(hk[grp], hc[grp], mask, w) - 1;
            }
            val = wave_seg_scan(val, q);
            if (wave_seg_tail(q, act) && val) atomicAdd((unsigned long long*)&c4v[ridx[q]], (unsigned long long)val);
        }
        accu = wave_sum(accu);
        if (lane_id() == 0 && accu) atomicAdd((unsigned long long*)&red[grp], (unsigned long long)accu);
        __syncthreads();
        if (valid && gt == 0 && red[grp]) atomicAdd((unsigned long long*)&c4v[u], (unsigned long long)red[grp]);
        __syncthreads();
    }
}

// Heavy tier: jobs (u, window) with u a vertex of large wedge count and the
// window a range of WS consecutive ranks for the wedge end w.  One 1024-thread
// workgroup per job counts the ends of u's wedges inside the window in dense
// LDS counters (16-bit halves of 32-bit words when every count fits 16 bits),
// so no global atomics touch the counts.  For every middle vertex v in N-(u)
// the wedge ends inside the window are one contiguous run of row v, found by
// two binary searches; the runs of 1024 middles at a time are flattened by a
// block scan and walked in contiguous per-thread chunks.  Pass A counts, pass
// B turns each count c into C(c, 2) for u and for w, pass C gives every middle
// v the sum of (c - 1) over its wedges.  Jobs are pulled from a device queue,
// largest vertices and highest windows first.
static constexpr int C4W_THREADS = 1024;
static constexpr int C4W_CHUNK = 16;
static constexpr int C4W_WORDS = 32768;  // 128 KiB of counters

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

// Computes the runs of middles c0 .. c0+1023 of u inside [W0, W1), keeps the
// non-empty ones in LDS (ridx base such that item t of run r sits at
// base[r] + t, middle vertex, first item) and the smallest and largest wedge
// end seen; returns the item count (run count in *nruns, rstart[nruns] = count).
// With a window table the run bounds are two table reads; otherwise two binary
// searches in the row.
template <bool TAB>
__device__ __forceinline__ i32 c4w_runs(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                        const i32* __restrict__ rpos, const i32* __restrict__ tab, i64 K1,
                                        i32 win, i64 b, i32 L, i32 c0, i32 W0, i32 W1, i64* rbase, i32* rmid,
                                        i32* rstart, i32* wsum, i32* stotal, i32* nruns, i32* wlo, i32* whi) {
    const i32 k = c0 + (i32)threadIdx.x;
    i32 len = 0;
    i64 s0 = 0;
    i32 v = 0;
    if (k < L) {
        v = ridx[b + k];
        const i64 rs = roff[v];
        const i32 cut = rpos[b + k];  // neighbours of v below u
        if (TAB) {
            const i32 a0 = tab[(i64)v * K1 + win];
            const i32 a1 = min(tab[(i64)v * K1 + win + 1], cut);
            s0 = rs + a0;
            len = a1 > a0 ? a1 - a0 : 0;
        } else {
            const i64 re = rs + cut;
            s0 = lower_bound_dev(ridx, rs, re, W0);
            len = (i32)(lower_bound_dev(ridx, s0, re, W1) - s0);
        }
    }
    if (len > 0) {
        atomicMin(wlo, ridx[s0]);
        atomicMax(whi, ridx[s0 + len - 1]);
    }
    const i32 pre = block_scan_1024(len, wsum, stotal);
    const i32 T = *stotal;
    __syncthreads();
    const i32 cidx = block_scan_1024(len > 0 ? 1 : 0, wsum, stotal);
    if (len > 0) {
        rbase[cidx] = s0 - pre;
        rmid[cidx] = v;
        rstart[cidx] = pre;
    }
    if (threadIdx.x == 0) {
        *nruns = *stotal;
        rstart[*stotal] = T;
    }
    __syncthreads();
    return T;
}

template <bool PACK16, bool TAB>
__global__ void __launch_bounds__(C4W_THREADS) k_c4_window(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                           const i32* __restrict__ lo, const i32* __restrict__ rpos,
                                                           const i32* __restrict__ tab, i64 K1,
                                                           const i32* __restrict__ heavy_sorted, u32 nheavy,
                                                           const i64* __restrict__ jobpre, u32* __restrict__ job_ctr,
                                                           i64* __restrict__ c4v) {
    constexpr i32 WS = PACK16 ? 2 * C4W_WORDS : C4W_WORDS;
    constexpr int NWV = C4W_THREADS / WAVE;
    __shared__ u32 cnt[C4W_WORDS];
    __shared__ i64 rbase[C4W_THREADS + 1];
    __shared__ i32 rmid[C4W_THREADS + 1];
    __shared__ i32 rstart[C4W_THREADS + 1];
    __shared__ i32 flags[NWV][WAVE];
    __shared__ i32 wsum[C4W_THREADS / WAVE];
    __shared__ i32 stotal, nruns, wlo, whi;
    __shared__ i64 sjob;
    __shared__ i64 red;
    const i64 njobs = jobpre[nheavy];
    const int wv = threadIdx.x / WAVE;
    const int l = lane_id();
    while (true) {
        if (threadIdx.x == 0) {
            sjob = (i64)atomicAdd(job_ctr, 1u);
            red = 0;
            wlo = 0x7fffffff;
            whi = -1;
        }
        __syncthreads();
        const i64 j = sjob;
        if (j >= njobs) break;
        // job j -> (heavy vertex, window), heaviest vertices first, top windows first
        const i64 h = last_le_dev(jobpre, 0, (i64)nheavy - 1, j);
        const i64 u = heavy_sorted[nheavy - 1 - h];
        const i64 nwin = jobpre[h + 1] - jobpre[h];
        const i32 win = (i32)(nwin - 1 - (j - jobpre[h]));
        const i32 W0 = win * WS;
        const i32 W1 = (i32)std::min<i64>((i64)W0 + WS, u);
        const i64 b = roff[u];
        const i32 L = lo[u];
        const bool one_chunk = L <= C4W_THREADS;
        i32 T = 0;
        if (one_chunk) {
            // all middles fit one chunk: runs first, then clear only the touched range
            T = c4w_runs<TAB>(roff, ridx, rpos, tab, K1, win, b, L, 0, W0, W1, rbase, rmid, rstart, wsum, &stotal,
                              &nruns, &wlo, &whi);
            if (T == 0) continue;  // T is block-uniform (LDS)
            const i32 q0 = PACK16 ? (wlo - W0) >> 1 : wlo - W0;
            const i32 q1 = PACK16 ? (whi - W0) >> 1 : whi - W0;
            for (i32 q = q0 + threadIdx.x; q <= q1; q += C4W_THREADS) cnt[q] = 0;
        } else {
            for (int q = threadIdx.x; q < C4W_WORDS; q += C4W_THREADS) cnt[q] = 0;
        }
        __syncthreads();
        // pass A: count the wedge ends in the window
        for (i32 c0 = 0; c0 < L; c0 += C4W_THREADS) {
            if (!one_chunk)
                T = c4w_runs<TAB>(roff, ridx, rpos, tab, K1, win, b, L, c0, W0, W1, rbase, rmid, rstart, wsum,
                                  &stotal, &nruns, &wlo, &whi);
            const i32 per = ((T + NWV * WAVE - 1) / (NWV * WAVE)) * WAVE;
            run_walk<4>(std::min(T, wv * per), std::min(T, (wv + 1) * per), rbase, rstart, nruns, flags[wv], ridx,
                        [&](bool act, i32, i32, i32 w, i64, u64) {
                            if (act) c4w_inc<PACK16>(cnt, w - W0);
                        });
            __syncthreads();
        }
        // pass B: C(c, 2) to u and to w, over the touched range only (empty when
        // no middle has a wedge end in the window: then whi < wlo)
        i64 accu = 0;
        const i32 xa = whi >= wlo ? wlo - W0 : 0;
        const i32 xb = whi >= wlo ? whi - W0 : -1;
        for (i32 x = xa + (i32)threadIdx.x; x <= xb; x += C4W_THREADS) {
            const i64 c = c4w_get<PACK16>(cnt, x);
            if (c >= 2) {
                const i64 pr = c * (c - 1) / 2;
                accu += pr;
                atomicAdd((unsigned long long*)&c4v[W0 + x], (unsigned long long)pr);
            }
        }
        accu = wave_sum(accu);
        if (l == 0 && accu) atomicAdd((unsigned long long*)&red, (unsigned long long)accu);
        // pass C: (c - 1) to the middle of every wedge; per-run sums from a wave
        // prefix sum and the run-start mask
        for (i32 c0 = 0; c0 < L; c0 += C4W_THREADS) {
            if (!one_chunk)
                T = c4w_runs<TAB>(roff, ridx, rpos, tab, K1, win, b, L, c0, W0, W1, rbase, rmid, rstart, wsum,
                                  &stotal, &nruns, &wlo, &whi);
            const i32 per = ((T + NWV * WAVE - 1) / (NWV * WAVE)) * WAVE;
            const i32 tb = std::min(T, (wv + 1) * per);
            run_walk<4>(std::min(T, wv * per), tb, rbase, rstart, nruns, flags[wv], ridx,
                     [&](bool act, i32 t, i32 r, i32 w, i64, u64 mask) {
                         i64 val = act ? (i64)c4w_get<PACK16>(cnt, w - W0) - 1 : 0;
                         // inclusive prefix over the wave
                         i64 P = val;
#pragma unroll
                         for (int o = 1; o < WAVE; o <<= 1) {
                             const i64 y = __shfl_up(P, o, WAVE);
                             if (l >= o) P += y;
                         }
                         const u64 below = mask & (l == WAVE - 1 ? ~0ull : ((1ull << (l + 1)) - 1));
                         const int sl = below ? 63 - __clzll((long long)below) : 0;  // first lane of my run
                         const i64 before = __shfl(P, sl > 0 ? sl - 1 : 0, WAVE);
                         const bool tail = act && (l == WAVE - 1 || ((mask >> (l + 1)) & 1ull) || t + 1 >= tb);
                         const i64 sum = P - (sl > 0 ? before : 0);
                         if (tail && sum) atomicAdd((unsigned long long*)&c4v[rmid[r]], (unsigned long long)sum);
                     });
            __syncthreads();
        }
        if (threadIdx.x == 0 && red) atomicAdd((unsigned long long*)&c4v[u], (unsigned long long)red);
        __syncthreads();
    }
}

// Window table: tab[v * K1 + k] = number of neighbours of v with rank below k * WS.
__global__ void k_c4_table(const i64* __restrict__ roff, const i32* __restrict__ ridx, i64 n, i64 K1, i64 WS,
                           i32* __restrict__ tab) {
    const i64 total = n * K1;
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (i64)gridDim.x * blockDim.x) {
        const i64 v = q / K1, k = q - v * K1;
        const i64 b = roff[v], e = roff[v + 1];
        const i64 key = k * WS;
        tab[q] = (i32)(key >= n ? e - b : lower_bound_dev(ridx, b, e, key) - b);
    }
}

__global__ void k_set_pair(i64* p, i64 a, i64 b) {
    p[0] = a;
    p[1] = b;
}

// Windows per heavy vertex, in descending vertex order.
__global__ void k_c4_jobs(const i32* __restrict__ heavy_sorted, u32 nheavy, i64 WS, i64* __restrict__ jobcnt) {
    for (i64 h = (i64)blockIdx.x * blockDim.x + threadIdx.x; h < nheavy; h += (i64)gridDim.x * blockDim.x) {
        const i64 u = heavy_sorted[nheavy - 1 - h];
        jobcnt[h] = (u + WS - 1) / WS;
    }
}

// ------------------------------------------------------------ finalize / net

__global__ void k_finalize(i64 n, const i32* __restrict__ rdeg, const i32* __restrict__ perm,
                           const i64* __restrict__ sumd, const i64* __restrict__ s7, const i64* __restrict__ c3v,
                           const i64* __restrict__ ap2, const i64* __restrict__ ac3, const i64* __restrict__ d10,
                           const i64* __restrict__ d14, const i64* __restrict__ d13, const i64* __restrict__ c4v,
                           const i64* __restrict__ k4v, i64* __restrict__ out, int net) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        const i64 d = rdeg[r];
        const i64 p2 = sumd[r] - d;
        const i64 c3 = c3v[r];
        i64 f[16];
        f[0] = 1;
        f[1] = d;
        f[2] = p2;
        f[3] = d * (d - 1) / 2;
        f[4] = c3;
        f[5] = ap2[r] - d * (d - 1) - 2 * c3;
        f[6] = p2 * (d - 1) - 2 * c3;
        f[7] = s7[r];
        f[8] = d * (d - 1) * (d - 2) / 6;
        f[9] = ac3[r] - 2 * c3;
        f[10] = d10[r];
        f[11] = (d - 2) * c3;
        f[12] = c4v[r];
        f[13] = d13[r];
        f[14] = d14[r];
        f[15] = k4v[r];
        if (d < 2) {  // every term is 0 there, (d - 1) and (d - 2) factors included
            f[3] = 0;
            f[6] = 0;
            f[8] = 0;
            f[11] = 0;
        }
        if (net) raw_to_net16(f);
        i64* o = out + (i64)perm[r] * 16;
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
            *(longlong2*)(o + k) = make_longlong2(f[k], f[k + 1]);
        }
    }
}

__global__ void k_net(i64 n, const i64* __restrict__ raw, i64* __restrict__ net) {
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        i64 f[16];
        const i64* src = raw + r * 16;
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
            const longlong2 x = *(const longlong2*)(src + k);
            f[k] = x.x;
            f[k + 1] = x.y;
        }
        raw_to_net16(f);
        i64* dst = net + r * 16;
#pragma unroll
        for (int k = 0; k < 16; k += 2) *(longlong2*)(dst + k) = make_longlong2(f[k], f[k + 1]);
    }
}

// ------------------------------------------------------------ launchers

hipError_t launch_l1(i64 n, i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_l1, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.rdeg, n, nnz, w.sumd,
                       w.s7);
    return hipGetLastError();
}

hipError_t launch_l2(i64 n, i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_l2, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.rdeg, w.C3, w.sumd,
                       w.c3v, n, nnz, w.ap2, w.ac3, w.d10, w.d14);
    return hipGetLastError();
}

hipError_t launch_fill_c3(i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_c3, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.rpos, nnz, w.C3);
    return hipGetLastError();
}

hipError_t launch_tri(i64 n, i64 nnz, RawWs& w, const DevPlan& hp, int mode, bool stored, hipStream_t s,
                      SegTimer& tm) {
    (void)nnz;
    const u32 c0 = hp.n_tri[0], c1 = hp.n_tri[1], c2 = hp.n_tri[2];
    const i32* l0 = w.tri_list;
    const i32* l1 = w.tri_list + n;
    const i32* l2 = w.tri_list + 2 * n;
    hipError_t e;
    if (mode == 1) {
        // triangle pass; the wave and LDS tiers also store their N+ bitmaps
        tm.mark(FGLT_SEG_TRI1_WAVE, s);
        if ((e = launch_tri1_stored(n, w, hp, stored, s, 0)) != hipSuccess) return e;
        tm.mark(FGLT_SEG_TRI1_LDS, s);
        if ((e = launch_tri1_stored(n, w, hp, stored, s, 1)) != hipSuccess) return e;
        tm.mark(FGLT_SEG_TRI1_GLOBAL, s);
        if (c2) hipLaunchKernelGGL((k_tri_block<1, true>), dim3(std::min<u32>(c2, NUM_TRI_SLOTS)), dim3(PT), 0, s,
                                   w.roff, w.ridx, w.lo, w.rdeg, w.G, l2, c2, w.C3, w.c3v, w.k4v, w.d13, w.tri_slots,
                                   w.tri_slot_words, w.plan);
    } else {
        // clique and diamond pass: from the stored bitmaps, or by scanning again
        tm.mark(FGLT_SEG_TRI2_WAVE, s);
        if (stored) {
            if ((e = launch_tri2_stored(n, w, hp, s, 0)) != hipSuccess) return e;
        } else if (c0) {
            hipLaunchKernelGGL((k_tri_wave<2>), dim3(grid_for(c0, 4, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.lo,
                               w.rdeg, w.G, l0, c0, w.C3, w.c3v, w.k4v, w.d13, w.plan);
        }
        tm.mark(FGLT_SEG_TRI2_LDS, s);
        if (stored) {
            if ((e = launch_tri2_stored(n, w, hp, s, 1)) != hipSuccess) return e;
        } else if (c1) {
            hipLaunchKernelGGL((k_tri_block<2, false>), dim3(grid_for(c1, 1, 65536)), dim3(PT), 0, s, w.roff,
                               w.ridx, w.lo, w.rdeg, w.G, l1, c1, w.C3, w.c3v, w.k4v, w.d13, w.tri_slots,
                               w.tri_slot_words, w.plan);
        }
        tm.mark(FGLT_SEG_TRI2_GLOBAL, s);
        if (c2) hipLaunchKernelGGL((k_tri_block<2, true>), dim3(std::min<u32>(c2, NUM_TRI_SLOTS)), dim3(PT), 0, s,
                                   w.roff, w.ridx, w.lo, w.rdeg, w.G, l2, c2, w.C3, w.c3v, w.k4v, w.d13, w.tri_slots,
                                   w.tri_slot_words, w.plan);
    }
    return hipGetLastError();
}

hipError_t launch_c4(i64 n, i64 nnz, RawWs& w, const DevPlan& hp, hipStream_t s, SegTimer& tm) {
    (void)nnz;
    const u32 c0 = hp.n_c4[0], c1 = hp.n_c4[1], c2 = hp.n_c4[2];
    tm.mark(FGLT_SEG_C4_WAVE, s);
    if (c0) hipLaunchKernelGGL((k_c4_hash<1, 256>), dim3(grid_for(c0, 4, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.lo,
                               w.G, w.c4_list, c0, w.c4v);
    tm.mark(FGLT_SEG_C4_BLOCK, s);
    if (c1) hipLaunchKernelGGL((k_c4_hash<4, 4096>), dim3(grid_for(c1, 1, 65536)), dim3(PT), 0, s, w.roff, w.ridx,
                               w.lo, w.G, w.c4_list + n, c1, w.c4v);
    tm.mark(FGLT_SEG_C4_HEAVY, s);
    if (c2) {
        // heavy vertices in ascending order, then (vertex, window) jobs
        i32* hs = w.c4_list + 2 * n;
        hipLaunchKernelGGL(k_set_pair, dim3(1), dim3(1), 0, s, w.c4_segoff, (i64)0, (i64)c2);
        hipError_t e = seg_sort(hs, w.c4_segoff, 1, bits_for_n(n), w.sort, 1, s);
        if (e != hipSuccess) return e;
        const bool pack16 = hp.d_max < 65536;
        const i64 WS = pack16 ? 2 * C4W_WORDS : C4W_WORDS;
        const i64 K1 = (n + WS - 1) / WS + 1;
        const bool use_tab = w.c4_tab != nullptr && n * K1 <= w.c4_tab_cap;
        if (use_tab)
            hipLaunchKernelGGL(k_c4_table, dim3(grid_for(n * K1, PT, 65536)), dim3(PT), 0, s, w.roff, w.ridx, n, K1,
                               WS, w.c4_tab);
        hipLaunchKernelGGL(k_c4_jobs, dim3(grid_for(c2, PT, 4096)), dim3(PT), 0, s, hs, c2, WS, w.c4_jobcnt);
        if ((e = scan_exclusive_i64(w.c4_jobcnt, w.c4_jobpre, c2, w.partials, s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(w.c4_jobctr, 0, sizeof(u32), s)) != hipSuccess) return e;
        const unsigned grid = 2048;
#define C4W_LAUNCH(P16, TB)                                                                                    \
    hipLaunchKernelGGL((k_c4_window<P16, TB>), dim3(grid), dim3(C4W_THREADS), 0, s, w.roff, w.ridx, w.lo, w.rpos, \
                       w.c4_tab, K1, hs, c2, w.c4_jobpre, w.c4_jobctr, w.c4v)
        if (pack16 && use_tab) C4W_LAUNCH(true, true);
        else if (pack16) C4W_LAUNCH(true, false);
        else if (use_tab) C4W_LAUNCH(false, true);
        else C4W_LAUNCH(false, false);
#undef C4W_LAUNCH
    }
    return hipGetLastError();
}

hipError_t launch_finalize(i64 n, RawWs& w, i64* out, bool net, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, w.rdeg, w.perm, w.sumd, w.s7, w.c3v,
                       w.ap2, w.ac3, w.d10, w.d14, w.d13, w.c4v, w.k4v, out, net ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_net(i64 n, const i64* raw, i64* net, hipStream_t s) {
    hipLaunchKernelGGL(k_net, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, raw, net);
    return hipGetLastError();
}

}  // namespace fglt
