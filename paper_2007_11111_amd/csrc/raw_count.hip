// raw_count.hip -- the counting passes of the transform, in rank space.
//
//   TRI mode 1:     oriented triangle listing per vertex u over N+(u); C3 on
//                   every oriented edge (C3 = A .* A^2, Lemma 2)
//   FILL:           C3 copied to the mirrored entries; row sums 2 c3 = C3 e, and row
//                   pass 1: sum_j d_j (-> p2 = A p1 - p1), sum_j C(d_j - 1, 2) (-> \hat d_7)
//   TRI mode 2:     the induced subgraph on N+(u) as LDS bitmaps; per vertex
//                   4-cliques (T e / 6, Section IV-C) and off-cord diamonds
//                   (D4,c e / 2) attributed to all four / three vertices
//   L2  row pass:   A p2, A c3, C3 (p1 - 2), sum_j C(C3(i,j), 2)   (Table I rows 5, 9, 10, 14),
//                   and the clique pass's per-entry shares stored at mirrored entries
//   C4:             (c4.hip) rank-ordered wedges u - v - w with v, w < u;
//                   4-cycles (C4,2 e / 2, Lemma 5) attributed to u, w and the middles
//   FINALIZE:       Table I assembled per vertex, Table II back-substitution,
//                   rows scattered back to the caller's vertex order
#include <algorithm>
#include <climits>

#include "walk.h"

namespace fglt {

static constexpr int PT = 256;


__device__ __forceinline__ void fence_agent() { __threadfence(); }


// ------------------------------------------------------------ row passes
//
// Entry-parallel passes that sum per-entry terms into their rows.  A
// wavefront takes RP_CH chunks of 64 consecutive entries, issues all their
// loads first, then sums each chunk's runs of equal rows (wave_runs /
// run_total) and adds the totals with one atomic per run and quantity.

static constexpr int RP_CH = 4;

template <class F>
__device__ __forceinline__ void row_chunks(i64 nnz, F&& f) {
    const i64 nw = ((i64)gridDim.x * blockDim.x) / WAVE;
    const int l = lane_id();
    for (i64 wv = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; wv * WAVE * RP_CH < nnz; wv += nw) {
        i64 p[RP_CH];
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) p[c] = wv * WAVE * RP_CH + c * WAVE + l;
        f(p);
    }
}

__device__ __forceinline__ void add_run(i64* acc, i32 r, i64 v, const WaveRuns& w) {
    const i64 t = run_total(v, w);
    if (w.tail && t) atomicAdd((unsigned long long*)&acc[r], (unsigned long long)t);
}

// After the clique pass: A p2, A c3, C3 (p1 - 2) and C(C3, 2) by rows
// (Table I rows 5, 9, 10, 14), and, when the clique pass stored per-entry
// counts (ek != nullptr), their row sums: it stores, for each N+ entry
// (u, v) of its wave and LDS tiers, the 4-cliques and diamonds it attributes
// to v, packed as dv << EK_SHIFT | kv, at the mirror (v, u).
__global__ void k_l2_rec(i64 n, const i32* __restrict__ rdeg, const i64* __restrict__ sumd,
                         const i64* __restrict__ c3x2, L2Rec* __restrict__ rec,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    for (i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (i64)gridDim.x * blockDim.x) {
        const i64 d = rdeg[v];
        rec[v] = L2Rec{sumd[v] - d, ((c3x2[v] >> 1) << 21) | d};
    }
}

__global__ void __launch_bounds__(PT) k_l2(const i32* __restrict__ rrow, const i32* __restrict__ ridx,
                                           const L2Rec* __restrict__ rec, const i32* __restrict__ C3,
                                           const i64* __restrict__ ek, i64 nnz, i64* __restrict__ ap2,
                                           i64* __restrict__ ac3, i64* __restrict__ d10, i64* __restrict__ d14,
                                           i64* __restrict__ k4v, i64* __restrict__ d13,
    const u32* __restrict__ storep, const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    if (!*storep) ek = nullptr;  // no per-entry clique counts without stored bitmaps
    row_chunks(nnz, [&](const i64* p) {
        i32 r[RP_CH], j[RP_CH], t[RP_CH];
        L2Rec g[RP_CH];
        i64 x[RP_CH];
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) {
            const i64 q = p[c] < nnz ? p[c] : nnz - 1;
            r[c] = rrow[q];
            j[c] = ridx[q];
            t[c] = C3[q];
            x[c] = ek ? ek[q] : 0;
        }
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) g[c] = rec[j[c]];
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) {
            const bool act = p[c] < nnz;
            const WaveRuns w = wave_runs(r[c], act);
            const i64 d = g[c].c3d & ((1 << 21) - 1), tt = act ? t[c] : 0;
            add_run(ap2, r[c], act ? g[c].p2 : 0, w);          // p2(j)
            add_run(ac3, r[c], act ? g[c].c3d >> 21 : 0, w);   // c3(j)
            add_run(d10, r[c], tt * (d - 2), w);              // C3(i,j) (p1(j) - 2); C3 = 0 when d_j = 1
            add_run(d14, r[c], tt * (tt - 1) / 2, w);         // C(C3(i,j), 2)
            if (ek) {
                const i64 xx = act ? x[c] : 0;
                add_run(k4v, r[c], xx & (((i64)1 << EK_SHIFT) - 1), w);
                add_run(d13, r[c], xx >> EK_SHIFT, w);
            }
        }
    });
}

// After the triangle pass: C3 of each N- entry copied from its mirror, the
// row sums C3 e = 2 c3 (each triangle at v lies on two of its edges;
// Lemma 2), and row pass 1 of Table I: A p1 and sum_j C(d_j - 1, 2).  When
// the clique pass stores per-entry counts, their slots are cleared here.
__global__ void __launch_bounds__(PT) k_fill_c3(const i64* __restrict__ mir, const i32* __restrict__ ridx,
                                                const i32* __restrict__ rrow, const i32* __restrict__ rdeg,
                                                i64 nnz, i32* __restrict__ C3, i64* __restrict__ c3x2,
                                                i64* __restrict__ sumd, i64* __restrict__ s7,
                                                i64* __restrict__ ek,
    const u32* __restrict__ storep,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    if (!*storep) ek = nullptr;  // no per-entry clique counts without stored bitmaps
    row_chunks(nnz, [&](const i64* p) {
        i32 r[RP_CH], j[RP_CH], cv[RP_CH], dj[RP_CH];
        bool lower[RP_CH];
        i64 src[RP_CH];
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) {
            const i64 q = p[c] < nnz ? p[c] : nnz - 1;
            r[c] = rrow[q];
            j[c] = ridx[q];
            lower[c] = j[c] < r[c];  // an N- entry takes its mirror's count, an N+ entry keeps its own
            src[c] = lower[c] ? mir[q] : q;
        }
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) {
            cv[c] = C3[src[c]];
            dj[c] = rdeg[j[c]];
        }
#pragma unroll
        for (int c = 0; c < RP_CH; ++c) {
            const bool act = p[c] < nnz;
            if (act && lower[c]) C3[p[c]] = cv[c];
            if (act && ek) ek[p[c]] = 0;
            const WaveRuns w = wave_runs(r[c], act);
            const i64 d = act ? dj[c] : 0;
            add_run(c3x2, r[c], act ? cv[c] : 0, w);
            add_run(sumd, r[c], d, w);                              // A p1
            add_run(s7, r[c], act ? (d - 1) * (d - 2) / 2 : 0, w);  // sum_j C(d_j - 1, 2)
        }
    });
}

// ------------------------------------------------------------ triangle / clique passes


// Wave tier: out-degree D in [2, 64]; one wavefront per vertex, 4 per block.
template <int MODE>
__global__ void __launch_bounds__(PT) k_tri_wave(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                 const i32* __restrict__ lo, const i32* __restrict__ rdeg,
                                                 const i64* __restrict__ G, const i32* __restrict__ list, const u32* __restrict__ countp,
                                                 i32* __restrict__ C3, i64* __restrict__ k4v,
                                                 i64* __restrict__ d13, DevPlan* plan,
    const u32* __restrict__ storep) {
    if (MODE == 2 && storep && *storep) return;  // the stored-bitmap kernels count instead
    const u32 count = *countp;  // the tier size, written on the device
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
                if (lane < D) {
                    const i32 c = sCnt[wid][lane];
                    if (c) atomicAdd(&C3[bu + lane], c);
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

// Triangle pass, out-degree above the hub tier's (the list's vertices with
// D > dmin): every vertex's items are cut into chunks of TRI_SPLIT_CH (jobs,
// numbered through the prefix jobpre over the list), which the workgroups take
// by grid stride, so that one vertex with many items keeps every workgroup
// busy.  An item (u, v_k, y), y in N+(v_k), is a triangle when y is in N+(u).
// N+(u) lies in the ranks above u: when they fit, a bitmap of them in LDS
// answers with one read, and a hit's position in N+(u) is its rank among the
// set bits (prefix counts per 8 words, then at most 8 word popcounts);
// otherwise a sample of at most TRI_SAMP entries of N+(u) in LDS narrows a
// search to one short stretch of the row.  Counts go to C3 with global
// atomics: the entries (u, y) and (v_k, y) one per hit, (u, v_k) one per run
// of lanes on the same entry.
static constexpr i64 TRI_SPLIT_CH = 262144;
static constexpr int TRI_SPLIT_T = 1024;  // threads per workgroup
static constexpr int TRI_SAMP = 4096;     // LDS sample entries
static constexpr int TRI_BITW = 24576;    // LDS bitmap words: ranks u + 1 .. u + 786432
static constexpr int TRI_ECAP = 4096;     // entries of a chunk held in LDS at a time

// Jobs per list entry (zero beyond the list and for out-degrees <= dmin).
__global__ void k_tri1_jobs(const i64* __restrict__ roff, const i32* __restrict__ lo, const i64* __restrict__ G,
                            const i32* __restrict__ list, const u32* __restrict__ countp, i64 dmin, i64 bound,
                            i64* __restrict__ jobcnt, const DevPlan* __restrict__ plan) {
    FGLT_GATE(&plan->err);
    const u32 count = *countp;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < bound; i += (i64)gridDim.x * blockDim.x) {
        i64 c = 0;
        if (i < (i64)count) {
            const i64 u = list[i];
            const i64 bu = roff[u] + lo[u];
            const i64 D = roff[u + 1] - bu;
            if (D > dmin) c = (G[bu + D] - G[bu] + TRI_SPLIT_CH - 1) / TRI_SPLIT_CH;
        }
        jobcnt[i] = c;
    }
}

// LDS of the out-neighbourhood lookup and of the staged entries, shared by
// the split triangle kernel and the clique kernel above the LDS tier.
struct NbrLds {
    u32 bits[TRI_BITW];      // bitmap of the ranks above u, or the sample (never both)
    i32 bpre[TRI_BITW / 8];  // set bits before each group of 8 words
    i32 eS[TRI_ECAP + 1];    // a block of a chunk's entries: their first items (from the chunk's start)
    i64 eB[TRI_ECAP];        // and where item t (from 0) of each sits: ridx[eB + t]
    i32 wsum[TRI_SPLIT_T / WAVE];
    i32 btot;
    i64 sq[2];
};
static_assert(TRI_SAMP <= TRI_BITW, "the sample shares the bitmap's memory");

// Positions in N+(u) = ridx[bu .. bu + D) (ascending ranks, all above u).
// When the ranks above u fit in the bitmap, a rank's position is its rank
// among the set bits: prefix counts per group of 8 words, then at most 8 word
// popcounts; otherwise every step-th entry of the row, in LDS, narrows a
// search to one stretch of at most step entries.
struct NbrLookup {
    i64 u, bu;
    i32 D;
    bool bm;
    i32 step, ns;
    __device__ NbrLookup(i64 u_, i64 bu_, i32 D_, i64 n) : u(u_), bu(bu_), D(D_) {
        bm = n - 1 - u <= 32 * (i64)TRI_BITW;
        step = 64 * ((D + 64 * TRI_SAMP - 1) / (64 * TRI_SAMP));
        ns = (D + step - 1) / step;
    }
    // Every thread of the (TRI_SPLIT_T-thread) workgroup; the caller
    // synchronises before the first find.
    __device__ void build(NbrLds& sm, const i32* __restrict__ ridx, i64 n) const {
        if (bm) {
            const i32 nw = (i32)((n - 1 - u + 31) >> 5);
            for (i32 q = threadIdx.x; q < nw; q += TRI_SPLIT_T) sm.bits[q] = 0;
            __syncthreads();
            for (i32 k = threadIdx.x; k < D; k += TRI_SPLIT_T) {
                const u32 r = (u32)(ridx[bu + k] - u - 1);
                atomicOr(&sm.bits[r >> 5], 1u << (r & 31));
            }
            __syncthreads();
            constexpr int GPT = TRI_BITW / 8 / TRI_SPLIT_T;  // groups of 8 words a thread
            const i32 ng = (nw + 7) >> 3;
            i32 gc[GPT], tsum = 0;
#pragma unroll
            for (int g = 0; g < GPT; ++g) {
                const i32 grp = (i32)threadIdx.x * GPT + g;
                i32 cg = 0;
                if (grp < ng)
#pragma unroll
                    for (int q = 0; q < 8; ++q) cg += grp * 8 + q < nw ? __popc(sm.bits[grp * 8 + q]) : 0;
                gc[g] = cg;
                tsum += cg;
            }
            i32 run = block_scan<TRI_SPLIT_T>(tsum, sm.wsum, &sm.btot);
#pragma unroll
            for (int g = 0; g < GPT; ++g) {
                sm.bpre[threadIdx.x * GPT + g] = run;
                run += gc[g];
            }
        } else {
            i32* const samp = reinterpret_cast<i32*>(sm.bits);
            for (i32 q = threadIdx.x; q < ns; q += TRI_SPLIT_T) samp[q] = ridx[bu + (i64)q * step];
        }
    }
    // Whether y (a rank above u) is in N+(u); pos = the entries of N+(u)
    // below y (its position there when it is), ascending with y.
    __device__ __forceinline__ bool locate(const NbrLds& sm, const i32* __restrict__ ridx, i32 y, i32& pos) const {
        if (bm) {
            const u32 r = (u32)(y - u - 1);
            const u32 wd = sm.bits[r >> 5];
            pos = sm.bpre[r >> 8] + __popc(wd & ((1u << (r & 31)) - 1u));
            for (u32 q = (r >> 8) << 3; q < (r >> 5); ++q) pos += __popc(sm.bits[q]);
            return (wd >> (r & 31)) & 1u;
        }
        const i32* const samp = reinterpret_cast<const i32*>(sm.bits);
        i32 a = 0, b = ns;  // the last sample entry <= y (entry 0 is below y)
        while (b - a > 1) {
            const i32 mid = (a + b) >> 1;
            if (samp[mid] <= y) a = mid;
            else b = mid;
        }
        const i64 lo_ = bu + (i64)a * step, hi_ = std::min<i64>(bu + D, lo_ + step);
        const i64 pp = lower_bound_dev(ridx, lo_, hi_, y);
        pos = (i32)(pp - bu);
        return pp < hi_ && ridx[pp] == y;
    }
};

// Items [t0, t1) of vertex u (t0 < t1 <= t0 + 2^31): entry q of u holds items
// [G[q] - gb, G[q+1] - gb), item t of it at ridx[roff[v] + lo[v] + t - (G[q] -
// gb)] with v = ridx[q].  Blocks of up to TRI_ECAP entries are staged in LDS
// side by side; the threads then take items tid, tid + 1024, ... of the
// block, each finding its entry by a search of the staged starts, and call
// f(q, e) with q the item's entry and e its position in ridx.  Lanes hold
// consecutive items, so a wavefront's entries are non-decreasing.  Every
// thread of the workgroup calls it.
template <class F>
__device__ __forceinline__ void walk_chunk(NbrLds& sm, const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                           const i32* __restrict__ lo, const i64* __restrict__ G, i64 bu, i32 D,
                                           i64 gb, i64 t0, i64 t1, F&& f) {
    if (threadIdx.x < WAVE) {  // the entries holding the first and the last item
        const i64 qa = wave_last_le(G + bu, D, gb + t0);
        const i64 qb = wave_last_le(G + bu, D, gb + t1 - 1);
        if (threadIdx.x == 0) {
            sm.sq[0] = qa;
            sm.sq[1] = qb;
        }
    }
    __syncthreads();
    const i64 qa = sm.sq[0], qb = sm.sq[1];
    for (i64 sa = qa; sa <= qb; sa += TRI_ECAP) {
        const i32 ne = (i32)std::min<i64>(TRI_ECAP, qb - sa + 1);
        for (i32 i = threadIdx.x; i < ne; i += TRI_SPLIT_T) {
            const i64 q = bu + sa + i;
            const i64 gs = G[q] - gb;
            const i32 v = ridx[q];
            sm.eB[i] = roff[v] + lo[v] - gs;
            sm.eS[i] = (i32)(std::max(gs, t0) - t0);
        }
        if (threadIdx.x == 0) sm.eS[ne] = (i32)(std::min(G[bu + sa + ne] - gb, t1) - t0);
        __syncthreads();
        const i32 ia = sm.eS[0], ib = sm.eS[ne];
        i32 cur = 0;
        for (i32 tr = ia + (i32)threadIdx.x; tr < ib; tr += TRI_SPLIT_T) {
            i32 ka = cur, kb = ne;  // eS[ka] <= tr < eS[kb] (ne: the end)
            while (kb - ka > 1) {
                const i32 mid = (ka + kb) >> 1;
                if (sm.eS[mid] <= tr) ka = mid;
                else kb = mid;
            }
            cur = ka;
            f(bu + sa + ka, sm.eB[ka] + t0 + tr);
        }
        __syncthreads();  // the next block of entries, or what follows the walk
    }
}

__global__ void __launch_bounds__(TRI_SPLIT_T) k_tri1_split(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                            const i32* __restrict__ lo, const i64* __restrict__ G,
                                                            const i32* __restrict__ list, const u32* __restrict__ countp,
                                                            const i64* __restrict__ jobpre, i64 n,
                                                            i32* __restrict__ C3, const DevPlan* __restrict__ plan) {
    FGLT_GATE(&plan->err);
    const u32 count = *countp;
    __shared__ NbrLds sm;
    __shared__ i64 s_vi;
    const i64 total = jobpre[count];
    i64 have = -1;  // the list entry whose lookup structure is in LDS
    for (i64 j = blockIdx.x; j < total; j += gridDim.x) {
        if (threadIdx.x < WAVE) {
            const i64 vi = wave_last_le(jobpre, (i64)count, j);
            if (threadIdx.x == 0) s_vi = vi;
        }
        __syncthreads();
        const i64 vi = s_vi;
        const i64 u = list[vi];
        const i64 bu = roff[u] + lo[u];
        const i32 D = (i32)(roff[u + 1] - bu);
        const NbrLookup nb(u, bu, D, n);
        if (vi != have) {
            nb.build(sm, ridx, n);
            have = vi;
        }
        const i64 gb = G[bu];
        const i64 T = G[bu + D] - gb;
        const i64 t0 = (j - jobpre[vi]) * TRI_SPLIT_CH, t1 = std::min<i64>(T, t0 + TRI_SPLIT_CH);
        walk_chunk(sm, roff, ridx, lo, G, bu, D, gb, t0, t1, [&](i64 q, i64 e) {
            i32 l;
            const bool hit = nb.locate(sm, ridx, ridx[e], l);
            if (hit) {
                atomicAdd(&C3[bu + l], 1);
                atomicAdd(&C3[e], 1);
            }
            wave_run_add(C3, q, hit);  // one add per run of lanes on entry q
        });
    }
}

__device__ __forceinline__ u64 readlane_u64(u64 v, int lane) {
    const u32 a = (u32)__builtin_amdgcn_readlane((int)(u32)v, lane);
    const u32 b = (u32)__builtin_amdgcn_readlane((int)(u32)(v >> 32), lane);
    return (u64)b << 32 | a;
}

// Calls f(p) for the set bits p of a row of words spread over the lanes
// (lane z holds word z0 + z: p = 64 (z0 + z) + bit), four at a time -- f gets
// up to 4 positions and their count -- so that the gathers f issues for them
// are in flight together.  Wave-uniform.
template <class F>
__device__ __forceinline__ void row_bits4(u64 word, i32 z0, F&& f) {
    u64 nz = __ballot(word != 0);
    u64 wd = 0;
    i32 base = 0;
    for (;;) {
        i32 p[4];
        int c = 0;
        while (c < 4) {
            if (!wd) {
                if (!nz) break;
                const int z = __ffsll((long long)nz) - 1;
                nz &= nz - 1;
                wd = readlane_u64(word, z);
                base = (z0 + z) * 64;
            }
            p[c++] = base + __ffsll((long long)wd) - 1;
            wd &= wd - 1;
        }
        if (c) f(p, c);
        if (c < 4) return;
    }
}

// Clique / diamond pass above the LDS tier with the bitmaps in device memory:
// the list's vertices with dmin < D <= dmax (dmin_nostore in place of dmin
// when the hub tier stored no bitmaps), one TRI_SPLIT_T-thread workgroup at a
// time, each with a slot of slot_words >= 2 D ceil(D / 64) words for B (row
// k: the positions l > k of N+(u) adjacent to v_k, the subgraph H that N+(u)
// induces) and C = B^T.  The items (u, v_k, y) are walked in chunks as in the
// split triangle kernel, with y's position l from the same LDS lookup; a hit
// sets B(k, l) (one atomic per word and run of lanes) and adds C3(v_k, y) - 1
// to u's diamonds, and C follows by 64 x 64 bit transposes.  Then one
// wavefront per row k, one word of the row per lane: the triangles of H
// through k number R + M + X with R = sum over l in B_k of |B_k & B_l| and
// M + X = sum over j in C_k of |B_j & (B_k | C_k)| (each a 4-clique with u
// and v_k; R summed over k counts u's own once), and v_k's diamonds add
// C3(u, v_x) - 1 for every x in B_k | C_k.  A lane reads B_l or B_j only
// where its own word of the row is non-zero and at or past the word of
// position l + 1 (j + 1), the first that B_l (B_j) can hold.
__global__ void __launch_bounds__(TRI_SPLIT_T) k_tri2_big(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                          const i32* __restrict__ lo, const i64* __restrict__ G,
                                                          const i32* __restrict__ list, const u32* __restrict__ countp,
                                                          i64 dmin, i64 dmax, i64 dmin_nostore, i64 n,
                                                          const i32* __restrict__ C3, i64* __restrict__ k4v,
                                                          i64* __restrict__ d13, u64* __restrict__ slots,
                                                          i64 slot_words, const DevPlan* __restrict__ plan,
                                                          const u32* __restrict__ storep) {
    FGLT_GATE(&plan->err);
    if (storep && !*storep) dmin = dmin_nostore;  // nothing stored: the hub tier's vertices too
    const u32 count = *countp;
    constexpr int NWV = TRI_SPLIT_T / WAVE;
    __shared__ NbrLds sm;
    __shared__ i64 red[2];
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    u64* const B = slots + (i64)blockIdx.x * slot_words;
    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const i32 D = (i32)(roff[u + 1] - bu);
        if (D <= dmin || D > dmax) continue;  // another launch takes it (uniform over the workgroup)
        const i32 W = (D + 63) >> 6;
        u64* const C = B + (i64)D * W;
        for (i64 q = threadIdx.x; q < 2 * (i64)D * W; q += TRI_SPLIT_T) B[q] = 0;
        if (threadIdx.x == 0) red[0] = red[1] = 0;
        const NbrLookup nb(u, bu, D, n);
        nb.build(sm, ridx, n);
        fence_agent();
        __syncthreads();
        fence_agent();
        const i64 gb = G[bu];
        const i64 T = G[bu + D] - gb;
        i64 d13u = 0;
        for (i64 t0 = 0; t0 < T; t0 += TRI_SPLIT_CH)
            walk_chunk(sm, roff, ridx, lo, G, bu, D, gb, t0, std::min<i64>(T, t0 + TRI_SPLIT_CH), [&](i64 q, i64 e) {
                i32 l;
                const bool hit = nb.locate(sm, ridx, ridx[e], l);
                if (hit) d13u += (i64)C3[e] - 1;
                if (__ballot(hit)) {
                    // lanes hold consecutive items: within one entry k the
                    // positions l ascend, so the hits bound for one word of
                    // row k sit in one run of lanes, whose bits (distinct,
                    // so their sum is their union) go in with one atomic
                    const i32 k = (i32)(q - bu);  // l > k: y follows v_k in rank
                    const WaveRuns wr = wave_runs(k * (W + 1) + (l >> 6), true);
                    const u64 bitsum = (u64)run_total(hit ? (i64)(1ull << (l & 63)) : 0, wr);
                    if (wr.tail && bitsum) atomicOr((unsigned long long*)&B[(i64)k * W + (l >> 6)], bitsum);
                }
            });
        fence_agent();
        __syncthreads();
        fence_agent();
        // C = B^T by 64 x 64 blocks (B holds bits l > k only: blocks on and
        // above the diagonal)
        for (i32 p = wv; p < W * W; p += NWV) {
            const i32 bi = p / W, bj = p - bi * W;
            if (bj < bi) continue;
            const i32 r = bi * 64 + lane, c = bj * 64 + lane;
            const u64 t = wave_transpose64(r < D ? B[(i64)r * W + bj] : 0ull);
            if (c < D) C[(i64)c * W + bi] = t;
        }
        fence_agent();
        __syncthreads();
        fence_agent();
        i64 Rsum = 0;
        for (i32 k = wv; k < D; k += NWV) {
            const u64* Bk = B + (i64)k * W;
            const u64* Ck = C + (i64)k * W;
            i64 R = 0, MX = 0, dv = 0;
            for (i32 z0 = 0; z0 < W; z0 += WAVE) {
                const i32 z = z0 + lane;  // this lane's word
                const u64 bk = z < W ? Bk[z] : 0ull, ck = z < W ? Ck[z] : 0ull;
                const u64 ak = bk | ck;
                FOR_BITS(ak, b, dv += (i64)C3[bu + z * 64 + b] - 1);
                if (!__ballot(ak != 0)) continue;
                // every set bit of the row (all its words) against this lane's word
                for (i32 y0 = 0; y0 < W; y0 += WAVE) {
                    const i32 y = y0 + lane;
                    const u64 rb = y0 == z0 ? bk : (y < W ? Bk[y] : 0ull);
                    const u64 rc = y0 == z0 ? ck : (y < W ? Ck[y] : 0ull);
                    row_bits4(rb, y0, [&](const i32* p, int c) {
                        u64 x[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            x[i] = i < c && bk && z >= ((p[i] + 1) >> 6) ? B[(i64)p[i] * W + z] : 0ull;
#pragma unroll
                        for (int i = 0; i < 4; ++i) R += __popcll(bk & x[i]);
                    });
                    row_bits4(rc, y0, [&](const i32* p, int c) {
                        u64 x[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            x[i] = i < c && ak && z >= ((p[i] + 1) >> 6) ? B[(i64)p[i] * W + z] : 0ull;
#pragma unroll
                        for (int i = 0; i < 4; ++i) MX += __popcll(ak & x[i]);
                    });
                }
            }
            R = wave_sum(R);
            MX = wave_sum(MX);
            dv = wave_sum(dv);
            if (lane == 0) {
                const i32 vk = ridx[bu + k];
                if (R + MX) atomicAdd((unsigned long long*)&k4v[vk], (unsigned long long)(R + MX));
                if (dv) atomicAdd((unsigned long long*)&d13[vk], (unsigned long long)dv);
                Rsum += R;
            }
        }
        d13u = wave_sum(d13u);
        if (lane == 0) {
            if (Rsum) atomicAdd((unsigned long long*)&red[0], (unsigned long long)Rsum);
            if (d13u) atomicAdd((unsigned long long*)&red[1], (unsigned long long)d13u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            if (red[0]) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)red[0]);
            if (red[1]) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)red[1]);
        }
        fence_agent();
        __syncthreads();  // the slot and the LDS are reused by the next vertex
        fence_agent();
    }
}

// Clique / diamond pass, LDS tier (64 < D <= TRI_LDS_MAX) when the triangle
// pass stored no bitmaps: one workgroup per vertex rebuilds B (and C = B^T)
// in LDS from the items (u, v_k, y), y's position in N+(u) by a search of
// the LDS copy of N+(u) past k, then counts as the kernel above the LDS tier
// does, one thread per row.
__global__ void __launch_bounds__(PT) k_tri2_block(const i64* __restrict__ roff, const i32* __restrict__ ridx,
                                                   const i32* __restrict__ lo, const i64* __restrict__ G,
                                                   const i32* __restrict__ list, const u32* __restrict__ countp,
                                                   const i32* __restrict__ C3, i64* __restrict__ k4v,
                                                   i64* __restrict__ d13, const u32* __restrict__ storep) {
    if (*storep) return;  // the clique pass from stored bitmaps has counted instead (device flag)
    const u32 count = *countp;  // the tier size, written on the device
    constexpr int DM = TRI_LDS_MAX;
    constexpr int WM = DM / 64;
    __shared__ i32 L[DM];
    __shared__ i32 Pre[DM + 1];
    __shared__ i64 Bv[DM];
    __shared__ i32 Cnt[DM];
    __shared__ u64 B[DM * WM];
    __shared__ u64 C[DM * WM];
    __shared__ i64 red[2];

    for (i64 it = blockIdx.x; it < (i64)count; it += gridDim.x) {
        const i64 u = list[it];
        const i64 bu = roff[u] + lo[u];
        const int D = (int)(roff[u + 1] - bu);
        const int W = (D + 63) / 64;
        const i64 gb = G[bu];
        const i32 T = (i32)(G[bu + D] - gb);  // at most D * TRI_LDS_MAX in this tier
        for (int k = threadIdx.x; k < D; k += blockDim.x) {
            const i32 v = ridx[bu + k];
            L[k] = v;
            Bv[k] = roff[v] + lo[v];
            Pre[k] = (i32)(G[bu + k] - gb);
            Cnt[k] = C3[bu + k];
        }
        for (int q = threadIdx.x; q < D * W; q += blockDim.x) {
            B[q] = 0;
            C[q] = 0;
        }
        if (threadIdx.x == 0) {
            Pre[D] = T;
            red[0] = 0;
            red[1] = 0;
        }
        __syncthreads();

        i64 d13u = 0;
        for (i32 t = threadIdx.x; t < T; t += blockDim.x) {
            const int k = (int)last_le_dev(Pre, 0, D - 1, t);
            const i64 e = Bv[k] + (t - Pre[k]);
            const i32 y = ridx[e];
            const int l = (int)lower_bound_dev(L, (i64)k + 1, (i64)D, y);
            if (l < D && L[l] == y) {
                atomicOr((unsigned long long*)&B[k * W + (l >> 6)], 1ull << (l & 63));
                atomicOr((unsigned long long*)&C[l * W + (k >> 6)], 1ull << (k & 63));
                d13u += (i64)C3[e] - 1;
            }
        }
        __syncthreads();

        i64 Rsum = 0;
        for (int k = threadIdx.x; k < D; k += blockDim.x) {
            const u64* Bk = B + k * W;
            const u64* Ck = C + k * W;
            i64 R = 0, M = 0, X = 0, dv = 0;
            for (int wa = 0; wa < W; ++wa) {
                FOR_BITS(Bk[wa], bb, {
                    const int l = wa * 64 + bb;
                    const u64* Bl = B + l * W;
                    for (int z = 0; z < W; ++z) R += __popcll(Bk[z] & Bl[z]);
                    dv += Cnt[l] - 1;
                });
                FOR_BITS(Ck[wa], bb, {
                    const int j = wa * 64 + bb;
                    const u64* Bj = B + j * W;
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
        __syncthreads();
        if (threadIdx.x == 0) {
            if (red[0]) atomicAdd((unsigned long long*)&k4v[u], (unsigned long long)red[0]);
            if (red[1]) atomicAdd((unsigned long long*)&d13[u], (unsigned long long)red[1]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ finalize / net

// Table I for rank-space vertex r from its degree and the accumulators.
// Orbits whose passes did not run read zeroed accumulators; a sub-dictionary
// leaves them out of its conversion and its output.
__device__ __forceinline__ void assemble_raw(i64 r, const i32* __restrict__ rdeg, const i64* __restrict__ sumd,
                                             const i64* __restrict__ s7, const i64* __restrict__ c3x2,
                                             const i64* __restrict__ ap2, const i64* __restrict__ ac3,
                                             const i64* __restrict__ d10, const i64* __restrict__ d14,
                                             const i64* __restrict__ d13, const i64* __restrict__ c4v,
                                             const i64* __restrict__ k4v, i64* f) {
    const i64 d = rdeg[r];
    const i64 p2 = sumd[r] - d;
    const i64 c3 = c3x2[r] >> 1;
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
}

__global__ void k_finalize(i64 n, const i32* __restrict__ rdeg, const i32* __restrict__ perm,
                           const i64* __restrict__ sumd, const i64* __restrict__ s7, const i64* __restrict__ c3x2,
                           const i64* __restrict__ ap2, const i64* __restrict__ ac3, const i64* __restrict__ d10,
                           const i64* __restrict__ d14, const i64* __restrict__ d13, const i64* __restrict__ c4v,
                           const i64* __restrict__ k4v, i64* __restrict__ out, int net,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        i64 f[16];
        assemble_raw(r, rdeg, sumd, s7, c3x2, ap2, ac3, d10, d14, d13, c4v, k4v, f);
        if (net) raw_to_net16(f);
        i64* o = out + (i64)perm[r] * 16;
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
            *(longlong2*)(o + k) = make_longlong2(f[k], f[k + 1]);
        }
    }
}

// A sub-dictionary with index set `mask` (Section V): the orbits of the set,
// raw or net by U16(s, s), scattered to caller order as [n][|s|].
__global__ void k_finalize_sub(i64 n, const i32* __restrict__ rdeg, const i32* __restrict__ perm,
                               const i64* __restrict__ sumd, const i64* __restrict__ s7, const i64* __restrict__ c3x2,
                               const i64* __restrict__ ap2, const i64* __restrict__ ac3, const i64* __restrict__ d10,
                               const i64* __restrict__ d14, const i64* __restrict__ d13, const i64* __restrict__ c4v,
                               const i64* __restrict__ k4v, i64* __restrict__ out, int net, unsigned mask, int ncols,
    const u32* __restrict__ errw) {
    FGLT_GATE(errw);
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
        i64 f[16];
        assemble_raw(r, rdeg, sumd, s7, c3x2, ap2, ac3, d10, d14, d13, c4v, k4v, f);
        if (net) raw_to_net_sub(f, mask);
        i64* o = out + (i64)perm[r] * ncols;
        int c = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if ((mask >> k) & 1u) o[c++] = f[k];
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

hipError_t launch_l2(i64 n, i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    const u32* const errw = &w.plan->err;
    hipLaunchKernelGGL(k_l2_rec, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, w.rdeg, w.sumd, w.c3x2, w.l2rec,
                       errw);
    hipLaunchKernelGGL(k_l2, dim3(grid_for(nnz, PT * RP_CH, 65536)), dim3(PT), 0, s, w.rrow, w.ridx, w.l2rec, w.C3,
                       w.ek, nnz, w.ap2, w.ac3, w.d10, w.d14, w.k4v, w.d13, (const u32*)&w.plan->stored, errw);
    return hipGetLastError();
}

hipError_t launch_fill_c3(i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_c3, dim3(grid_for(nnz, PT * RP_CH, 65536)), dim3(PT), 0, s, w.mir, w.ridx, w.rrow,
                       w.rdeg, nnz, w.C3, w.c3x2, w.sumd, w.s7, w.ek, (const u32*)&w.plan->stored,
                       (const u32*)&w.plan->err);
    return hipGetLastError();
}

hipError_t launch_tri(i64 n, i64 nnz, RawWs& w, int mode, i64 hub_max, hipStream_t s, SegTimer& tm) {
    const u32* const cnt = w.plan->n_tri;
    const u32* const stp = &w.plan->stored;
    const i32* l0 = w.tri_list;
    const i32* l1 = w.tri_list + n;
    const i32* l2 = w.tri_list + 2 * n;
    // the last tier's bound: vertices of out-degree above the LDS tier's.  The
    // clique pass shares out the global-bitmap slots' memory by the largest
    // out-degree a launch takes: out-degree up to TRI_MID_D, then ranges of
    // doubling out-degree, each launch with slots for its own largest bitmaps
    const i64 region = (i64)w.tri_nslots * w.tri_slot_words;
    i64 dplus = 1;  // above every out-degree (the degree order keeps them below sqrt(nnz))
    while (dplus * dplus <= nnz) ++dplus;
    const i64 tier_bound = std::min<i64>(n, nnz / (2 * TRI_LDS_MAX) + 1);
    auto slots_for = [&](i64 words, i64 cap) {
        return (unsigned)std::max<i64>(1, std::min<i64>({tier_bound, region / words, cap}));
    };
    const i64 d_mid = std::min<i64>(TRI_MID_D, dplus);
    hipError_t e;
    if (mode == 1) {
        // triangle pass; the wave, LDS and hub tiers also store their N+ bitmaps
        tm.mark(FGLT_SEG_TRI1_WAVE, s);
        if ((e = launch_tri1_stored(n, nnz, w, s, 0, hub_max)) != hipSuccess) return e;
        tm.mark(FGLT_SEG_TRI1_LDS, s);
        if ((e = launch_tri1_stored(n, nnz, w, s, 1, hub_max)) != hipSuccess) return e;
        tm.mark(FGLT_SEG_TRI1_GLOBAL, s);
        if ((e = launch_tri1_stored(n, nnz, w, s, 2, hub_max)) != hipSuccess) return e;
        // the rest of the last tier, split into chunks of items (the job
        // prefix over the list's n entries at most -- a plan with lower tier
        // bounds may put any vertex there -- with scan partials of its own:
        // the 4-cycle setup may scan on the second stream meanwhile)
        hipLaunchKernelGGL(k_tri1_jobs, dim3(grid_for(n + 1, PT, 4096)), dim3(PT), 0, s, w.roff, w.lo, w.G, l2,
                           cnt + 2, hub_max, n + 1, w.tri_jobpre, (const DevPlan*)w.plan);
        if ((e = scan_exclusive_i64(w.tri_jobpre, w.tri_jobpre, n + 1, w.tri_partials, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tri1_split, dim3(4 * 256), dim3(TRI_SPLIT_T), 0, s, w.roff, w.ridx, w.lo, w.G, l2,
                           cnt + 2, (const i64*)w.tri_jobpre, n, w.C3, (const DevPlan*)w.plan);
    } else {
        // clique and diamond pass: from the stored bitmaps, or by scanning
        // again (the stored flag is read on the device; each kernel of the
        // other way leaves at once)
        tm.mark(FGLT_SEG_TRI2_WAVE, s);
        if ((e = launch_tri2_stored(n, nnz, w, s, 0, hub_max)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_tri_wave<2>), dim3(grid_for(n, 4, 65536)), dim3(PT), 0, s, w.roff, w.ridx, w.lo, w.rdeg,
                           w.G, l0, cnt + 0, w.C3, w.k4v, w.d13, w.plan, stp);
        tm.mark(FGLT_SEG_TRI2_LDS, s);
        if ((e = launch_tri2_stored(n, nnz, w, s, 1, hub_max)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_tri2_block, dim3(grid_for(std::min<i64>(n, nnz / (2 * TRI_WAVE_MAX) + 1), 1, 65536)),
                           dim3(PT), 0, s, w.roff, w.ridx, w.lo, w.G, l1, cnt + 1, w.C3, w.k4v, w.d13, stp);
        tm.mark(FGLT_SEG_TRI2_GLOBAL, s);
        // the hub tier from its stored rows; the rest of the last tier (all of
        // it when nothing is stored) with bitmaps in the workspace
        if ((e = launch_tri2_stored(n, nnz, w, s, 2, hub_max)) != hipSuccess) return e;
        // out-degree ranges (hub_max, d_mid], (d_mid, 2 d_mid], (2 d_mid, 4 d_mid], ...,
        // each with as many slots for its largest bitmaps as the memory holds
        // (up to 256 workgroups: one per CU, the kernel's LDS allows no more)
        for (i64 a = hub_max, b = d_mid, first = 1;; a = b, b *= 2, first = 0) {
            const i64 top = std::min(b, dplus);
            const i64 words = 2 * top * ceil_div(top, 64);
            hipLaunchKernelGGL(k_tri2_big, dim3(slots_for(words, 256)), dim3(TRI_SPLIT_T), 0, s, w.roff, w.ridx,
                               w.lo, w.G, l2, cnt + 2, a, b >= dplus ? (i64)INT_MAX : b, first ? (i64)0 : a, n,
                               w.C3, w.k4v, w.d13, w.tri_slots, words, (const DevPlan*)w.plan, stp);
            if (b >= dplus) break;
            tm.note("tri2_global (an out-degree range)", s);
        }
    }
    return hipGetLastError();
}

// Six times the triangles of the graph (the sum over vertices of 2 c3) into
// plan->triangles (statistics only: one atomic per workgroup).
__global__ void __launch_bounds__(PT) k_count_triangles(i64 n, const i64* __restrict__ c3x2, DevPlan* plan) {
    FGLT_GATE(&plan->err);
    __shared__ i64 part[PT / WAVE];
    i64 sum = 0;
    for (i64 r = (i64)blockIdx.x * PT + threadIdx.x; r < n; r += (i64)gridDim.x * PT) sum += c3x2[r];
    sum = wave_sum(sum);
    if (lane_id() == 0) part[threadIdx.x / WAVE] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        i64 t = 0;
        for (int k = 0; k < PT / WAVE; ++k) t += part[k];
        if (t) atomicAdd((unsigned long long*)&plan->triangles, (unsigned long long)t);
    }
}

// Work counts of the byte model (statistics only, FGLT_WORKMODEL), one
// thread per oriented edge u -> v (an N+ entry of row u):
//   min_sum  += d(u)                  (the edge's share of sum_E min(d_i, d_j):
//                                      under the degree order d(u) <= d(v))
//   k4_merge += |T|^2 + sum_{w in T} d+(w),  T = N+(u) & N+(v)
// i.e. for every oriented triangle u < v < w the merge of the candidate set
// T with the out-list of w, the step count of an oriented 4-clique listing.
// T is found by walking the shorter out-list and searching the longer one.
__global__ void __launch_bounds__(PT) k_work_model(const i32* __restrict__ rrow, const i32* __restrict__ ridx,
                                                   const VRec* __restrict__ vrec, i64 nnz, DevPlan* plan) {
    FGLT_GATE(&plan->err);
    __shared__ i64 part[PT / WAVE];
    i64 ms = 0, ko = 0;
    for (i64 p = (i64)blockIdx.x * PT + threadIdx.x; p < nnz; p += (i64)gridDim.x * PT) {
        const i32 u = rrow[p], v = ridx[p];
        if (v <= u) continue;
        const VRec ru = vrec[u], rv = vrec[v];
        ms += ru.deg;
        i64 ab = ru.off + ru.lo, ae = ru.off + ru.deg;  // N+(u)
        i64 bb = rv.off + rv.lo, be = rv.off + rv.deg;  // N+(v)
        if (ae - ab > be - bb) {
            const i64 t0 = ab, t1 = ae;
            ab = bb;
            ae = be;
            bb = t0;
            be = t1;
        }
        i64 cnt = 0, sdp = 0;
        for (i64 q = ab; q < ae; ++q) {
            const i32 w = ridx[q];
            const i64 x = lower_bound_dev(ridx, bb, be, w);
            bb = x;  // both lists ascend
            if (x < be && ridx[x] == w) {
                const VRec rw = vrec[w];
                ++cnt;
                sdp += rw.deg - rw.lo;
            }
        }
        ko += cnt * cnt + sdp;
    }
    ms = block_sum<PT>(ms, part);
    ko = block_sum<PT>(ko, part);
    if (threadIdx.x == 0) {
        if (ms) atomicAdd((unsigned long long*)&plan->min_sum, (unsigned long long)ms);
        if (ko) atomicAdd((unsigned long long*)&plan->k4_merge, (unsigned long long)ko);
    }
}

hipError_t launch_work_model(i64 nnz, RawWs& w, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_work_model, dim3(grid_for(nnz, PT, 65536)), dim3(PT), 0, s, w.rrow, w.ridx, w.vrec, nnz,
                       w.plan);
    return hipGetLastError();
}

hipError_t launch_count_triangles(i64 n, RawWs& w, hipStream_t s) {
    const hipError_t e = fill_u32(&w.plan->triangles, 2, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_triangles, dim3(grid_for(n, PT, 256)), dim3(PT), 0, s, n, w.c3x2, w.plan);
    return hipGetLastError();
}

hipError_t launch_finalize(i64 n, RawWs& w, i64* out, bool net, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, w.rdeg, w.perm, w.sumd, w.s7, w.c3x2,
                       w.ap2, w.ac3, w.d10, w.d14, w.d13, w.c4v, w.k4v, out, net ? 1 : 0, (const u32*)&w.plan->err);
    return hipGetLastError();
}

hipError_t launch_finalize_sub(i64 n, RawWs& w, i64* out, bool net, unsigned mask, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_sub, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, w.rdeg, w.perm, w.sumd, w.s7,
                       w.c3x2, w.ap2, w.ac3, w.d10, w.d14, w.d13, w.c4v, w.k4v, out, net ? 1 : 0, mask,
                       __builtin_popcount(mask), (const u32*)&w.plan->err);
    return hipGetLastError();
}

hipError_t launch_net(i64 n, const i64* raw, i64* net, hipStream_t s) {
    hipLaunchKernelGGL(k_net, dim3(grid_for(n, PT, 65536)), dim3(PT), 0, s, n, raw, net);
    return hipGetLastError();
}

}  // namespace fglt
