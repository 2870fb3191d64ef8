// raw.h -- internal interface of the single-graph transform pipeline.
//
// All counting runs in "rank space": vertices relabelled by non-decreasing
// degree (ties by original id), rows re-sorted.  In rank space the degree
// orientation u -> v (v > u) of the triangle and clique passes is "later in
// the row", every row splits into N-(u) (entries < u) followed by N+(u)
// (entries > u), and the 4-cycle pass can stop each wedge scan at u.
#pragma once

#include "common.h"

namespace fglt {

// Tier thresholds.
constexpr int TRI_WAVE_MAX = 64;     // out-degree handled by one wavefront (one bitmap word)
constexpr int TRI_LDS_MAX = 512;     // out-degree whose bitmaps fit a workgroup's LDS
constexpr int TRI_HUB_MAX = 1088;    // out-degree of the hub tier: position map in LDS, and in the
                                     // clique pass A = B | B^T (1088 x 17 words, 145 KiB) in LDS
// Clique-pass count of an N+ entry, packed as dv << EK_SHIFT | kv: kv (the
// 4-cliques) is at most 2 (D - 1)^2 < 2^20 for D <= TRI_LDS_MAX, dv (the
// diamonds) below D * 2^21 (degrees < 2^21), so the word stays below 2^50.
constexpr int EK_SHIFT = 20;
// (the hub tier stores kv = C(D - 1, 2) at most)
static_assert(2 * (TRI_LDS_MAX - 1) * (TRI_LDS_MAX - 1) < (1 << EK_SHIFT), "kv must fit below EK_SHIFT");
static_assert((TRI_HUB_MAX - 1) * (TRI_HUB_MAX - 2) / 2 < (1 << EK_SHIFT), "hub kv must fit below EK_SHIFT");
constexpr int C4_WAVE_MAX = 128;     // wedges handled by one wavefront (256-slot LDS hash)
constexpr int C4_BLOCK_MAX = 2048;   // wedges handled by one workgroup (4096-slot LDS hash)
constexpr int C4_HASH_MAX = 16384;   // wedges handled by one large workgroup (32768-slot packed hash)
constexpr int TRI_MID_D = 4096;      // clique tier above the hub tier: out-degree bound of its first launch (then doubling)
constexpr int NUM_TRI_SLOTS = 64;    // clique pass above the hub tier: at most this many slots of the largest bitmaps
constexpr i64 C4W_SPAN = 65536;      // ranks per window of the 4-cycle window tier with 16-bit counts
constexpr int C4W_GRID = 256;        // workgroups of the 4-cycle window tier (one per CU)
constexpr int C4W_GROUP = 16;        // windows per job of a many-middle vertex when runs are searched

// Device statistics / plan words (one small block of device memory).
struct DevPlan {
    u32 err;
    u32 pad0;
    i64 d_max;
    i64 dplus_max;
    i64 sum_lo;
    i64 tri_items;
    i64 wedge_items;
    u32 n_tri[3];  // wave, lds, global tiers
    u32 n_c4[4];   // wave, block, hash, window tiers
    i64 tri_items_tier[3];
    i64 wedge_items_tier[4];
    i64 triangles;
    i64 c4_etab;  // entries of the window tier's per-entry window table (16-bit part)
    u32 n_c4_heavy; // window-tier vertices of degree >= 65536 (32-bit counters; the last ranks)
    u32 pad1;
    i64 n_low;      // vertices of degree <= 1 (the first ranks)
    u32 stored;     // the wave, LDS and hub tiers' bitmaps fit the workspace (and the clique pass runs)
    u32 use_etab;   // the window tier's per-entry table fits the workspace (and is wanted)
    i64 min_sum;  // byte model (FGLT_WORKMODEL): sum over edges of min(d_i, d_j)
    i64 k4_merge; // byte model: oriented 4-clique merge steps
};

// Per-vertex record of rank space, read with one 16-byte load where a kernel
// needs a neighbour's row: its start, |N-(v)| and degree.
struct __align__(16) VRec {
    i64 off;
    i32 lo;
    i32 deg;
};

// What row pass 2 gathers of a neighbour j, in one 16-byte load: p2(j), and
// c3(j) << 21 | d(j) (degrees are below 2^21, so c3 < 2^41 and the word < 2^62).
struct __align__(16) L2Rec {
    i64 p2;
    i64 c3d;
};

struct RawWs {
    // rank space structure
    i32* deg;     // [n] degrees, original order
    i32* perm;    // [n] rank -> original id
    i32* rank;    // [n] original id -> rank
    i32* rdeg;    // [n] degree by rank
    i32* lo;      // [n] |N-(u)|
    i64* cntd;    // [n+2] scratch of the degree sort
    i64* roff;    // [n+1]
    VRec* vrec;   // [n] roff, lo and degree of each vertex
    L2Rec* l2rec; // [n] p2, c3 and degree of each vertex, for row pass 2
    i32* ridx;    // [nnz]
    i32* rrow;    // [nnz] row of each entry (rank space)
    i32* rpos;    // [nnz] N- entry (u, v): position of u in row v; -1 for N+ entries
    i64* mir;     // [nnz] position of each entry's mirror (v, u)
    i64* G;       // [nnz+1] exclusive scan of per-entry work counts
    i32* C3;      // [nnz] triangle count per directed entry
    i64* ek;      // [max(nnz, n)] clique pass: packed 4-clique / diamond counts of the N+ entry (u, v)
                  // stored at its mirror (v, u); shares memory with sort.tmp (relabelling only)
    // per-vertex accumulators (rank space), contiguous block of 10*n; c3x2 = 2 c3
    i64* acc;
    i64 *sumd, *s7, *c3x2, *ap2, *ac3, *d10, *d14, *d13, *c4v, *k4v;
    // work lists
    i32* tri_list;  // [3][n]
    i32* c4_list;   // [4][n]
    // heavy-tier scratch
    u64* tri_slots;     // tri_nslots * tri_slot_words
    i64 tri_slot_words;
    int tri_nslots;     // slots of the largest bitmaps in that memory, 1..NUM_TRI_SLOTS (launches cut it finer)
    i64* tri_jobpre;    // [n+2] job counts, then their prefix, of the split triangle tier
    i64* tri_partials;  // scan partials of the triangle pass (the second stream scans with `partials`)
    i64* c4_segoff;     // [2] one segment over the window-tier list
    i64* c4_jobcnt;     // [n+1] jobs per window-tier vertex, then the prefix of their middle counts
    i64* c4_jobpre;     // [n+1] their exclusive scan
    i64* c4_ebase;      // [n+1] start of each window-tier vertex's block of the per-entry window table
    i64* c4_hjobcnt;    // [nnz/65536 + 2] jobs per window-tier vertex of degree >= 65536
    i64* c4_hjobpre;    // [nnz/65536 + 2] their exclusive scan
    u32* c4_jobctr;     // [4] job queue heads: window tier (16-bit, 32-bit counters), hash tier
    i64* bcnt;          // [n] bitmap words per vertex (clique pass store)
    i64* boff;          // [n+1] their exclusive scan
    u64* bstore;        // stored N+ bitmaps of the wave and LDS tiers
    i64 bstore_cap;     // its capacity in words
    u16* c4_tab;        // vertex window table of the window tier, 16-bit entries (optional)
    i64 c4_tab_cap;     // its capacity in entries
    u32* c4_scr;        // [C4W_GRID * c4_scr_cap] per-workgroup copies of a window's wedge ends
    i64 c4_scr_cap;
    // scratch
    i64* partials;
    SegSortWs sort;
    i64* rx_hist;       // radix sort: digit counts per tile, then their offsets
    DevPlan* plan;
};

RawWs carve_raw(Carver& c, i64 n, i64 nnz);

// The single-graph transform behind fglt_raw (api.hip).  With one_stream the
// 4-cycle pass's setup runs on `stream` too, so no second stream is created.
int raw_run(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices, int64_t* out, void* ws,
            size_t ws_bytes, unsigned flags, const fglt_raw_plan* plan, fglt_stats* stats, void* stream,
            bool one_stream);

// prep (raw_prep.hip)
hipError_t launch_check_input(i64 n, i64 nnz, const i64* off, const i32* idx, RawWs& w, hipStream_t s);
hipError_t launch_rank_and_relabel(i64 n, i64 nnz, const i64* off, const i32* idx, RawWs& w, hipStream_t s);
struct Tiers {
    i64 tri_wave, tri_lds, tri_hub, c4_wave, c4_block, c4_hash;
    i64 c4_hash_lmax;  // largest |N-(u)| whose counts fit the packed hash words
    int c4_rows;       // window tier's row cuts: 0 per-entry table where it fits, 1 per-vertex table, 2 searches
    int c4_group;      // window tier's windows per job of a many-middle vertex: 0 by the tier's size, else exactly
};
Tiers tiers_from_plan(const fglt_raw_plan* plan, i64 n);
int bits_for_n(i64 n);   // bits of the largest rank n - 1 (0 for n <= 1)
hipError_t launch_structure(i64 n, i64 nnz, RawWs& w, const Tiers& t, bool with_c4, bool want_store, int rows_mode,
                            hipStream_t s);

// counting (raw_count.hip)
// Optional event marks between launches (FGLT_TIMING) and progress lines
// (FGLT_PROGRESS: a host function on the stream prints a step's end on
// stderr when the stream gets there).
void progress_line(void* what);  // what: a static C string
extern const char* const kSegNames[FGLT_NSEG];
struct SegTimer {
    hipEvent_t ev[FGLT_NSEG + 1] = {};
    bool on = false;
    bool progress = false;
    int last = -1;
    // records the start of segment `seg` (and thereby the end of the previous one)
    void mark(int seg, hipStream_t s) {
        if (progress && last >= 0) note(kSegNames[last], s);
        if (on) (void)hipEventRecord(ev[seg], s);
        last = seg;
    }
    void note(const char* what, hipStream_t s) const {
        if (progress) (void)hipLaunchHostFunc(s, progress_line, const_cast<char*>(what));
    }
};

// tri.hip
hipError_t launch_bitmap_offsets(i64 n, RawWs& w, i64 lds_max, hipStream_t s);
hipError_t launch_tri1_stored(i64 n, i64 nnz, RawWs& w, hipStream_t s, int tier, i64 hub_max);
hipError_t launch_tri2_stored(i64 n, i64 nnz, RawWs& w, hipStream_t s, int tier, i64 hub_max);
hipError_t launch_tri(i64 n, i64 nnz, RawWs& w, int mode, i64 hub_max, hipStream_t s, SegTimer& tm);
hipError_t launch_fill_c3(i64 nnz, RawWs& w, hipStream_t s);
hipError_t launch_l2(i64 n, i64 nnz, RawWs& w, hipStream_t s);
hipError_t launch_c4_early(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s);
hipError_t launch_c4_etab(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s);
hipError_t launch_c4_late(i64 n, i64 nnz, RawWs& w, int rows_mode, int win_group, hipStream_t s, SegTimer& tm);
hipError_t launch_finalize(i64 n, RawWs& w, i64* out, bool net, hipStream_t s);
hipError_t launch_finalize_sub(i64 n, RawWs& w, i64* out, bool net, unsigned mask, hipStream_t s);
hipError_t launch_count_triangles(i64 n, RawWs& w, hipStream_t s);
hipError_t launch_work_model(i64 nnz, RawWs& w, hipStream_t s);
hipError_t launch_net(i64 n, const i64* raw, i64* net, hipStream_t s);

// Conversion raw -> net (Table II): back-substitution with U16.
__device__ __forceinline__ void raw_to_net16(i64* f) {
    // f arrives holding raw counts; solve U16 f = raw from the last row up.
    f[14] -= 3 * f[15];
    f[13] -= 3 * f[15];
    f[12] -= f[13] + f[14] + 3 * f[15];
    f[11] -= 2 * f[14] + 3 * f[15];
    f[10] -= 2 * f[13] + 2 * f[14] + 6 * f[15];
    f[9] -= 2 * f[13] + 3 * f[15];
    f[8] -= f[11] + f[14] + f[15];
    f[7] -= f[9] + f[10] + 2 * f[13] + f[14] + 3 * f[15];
    f[6] -= f[10] + 2 * f[11] + 2 * f[12] + 2 * f[13] + 4 * f[14] + 6 * f[15];
    f[5] -= 2 * f[9] + f[10] + 2 * f[12] + 4 * f[13] + 2 * f[14] + 6 * f[15];
    f[3] -= f[4];
    f[2] -= 2 * f[4];
}

// The conversion of a sub-dictionary with index set s (bit k = orbit k):
// U16(s, s) f_s = raw_s, the sub-matrix of Table II on s (Section V).  The
// orbits outside s are held at zero and never updated, so every row of the
// back-substitution reads only the orbits of s.
__device__ __forceinline__ void raw_to_net_sub(i64* f, unsigned s) {
#define IN(k) ((s >> (k)) & 1u)
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (!IN(k)) f[k] = 0;
    if (IN(14)) f[14] -= 3 * f[15];
    if (IN(13)) f[13] -= 3 * f[15];
    if (IN(12)) f[12] -= f[13] + f[14] + 3 * f[15];
    if (IN(11)) f[11] -= 2 * f[14] + 3 * f[15];
    if (IN(10)) f[10] -= 2 * f[13] + 2 * f[14] + 6 * f[15];
    if (IN(9)) f[9] -= 2 * f[13] + 3 * f[15];
    if (IN(8)) f[8] -= f[11] + f[14] + f[15];
    if (IN(7)) f[7] -= f[9] + f[10] + 2 * f[13] + f[14] + 3 * f[15];
    if (IN(6)) f[6] -= f[10] + 2 * f[11] + 2 * f[12] + 2 * f[13] + 4 * f[14] + 6 * f[15];
    if (IN(5)) f[5] -= 2 * f[9] + f[10] + 2 * f[12] + 4 * f[13] + 2 * f[14] + 6 * f[15];
    if (IN(3)) f[3] -= f[4];
    if (IN(2)) f[2] -= 2 * f[4];
#undef IN
}

}  // namespace fglt
