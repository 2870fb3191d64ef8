/*
 * fglt.h -- C ABI of the MI355X (gfx950) fast graphlet transform library.
 *
 * The library computes, for every vertex v of a simple undirected graph, the
 * frequencies of the 16 graphlet orbits sigma_0 .. sigma_15 on up to four
 * vertices (the dictionary Sigma_16 of Floros, Pitsianis and Sun, "Fast
 * Graphlet Transform of Sparse Graphs", Fig. 1 and Table I):
 *   - raw frequencies  \hat f(v) by the sparse matrix-vector formulas of
 *     Table I (Sections III and IV), and
 *   - net frequencies  f(v) = U16^{-1} \hat f(v) with the conversion matrix
 *     U16 of Table II (Section V), i.e. induced-subgraph orbit counts.
 *
 * Conventions for every entry point
 *   - Vertices are 0-based (the paper numbers them from 1).
 *   - Output arrays are n x 16 int64, row-major: row v, column k = sigma_k in
 *     the order of Table I.
 *   - All array arguments are DEVICE pointers unless marked (host); the caller
 *     allocates and frees every buffer (inputs, outputs, workspace). The
 *     library keeps no device allocation between calls, except cached HIP
 *     graphs of fglt_batch, released by fglt_batch_release().
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is enqueued
 *     on it; where an entry point synchronizes with that stream it says so.
 *   - Return value: FGLT_OK or a negative fglt_status; nothing throws across
 *     the ABI.  Argument checks happen on the host before any launch; errors
 *     reported by the HIP runtime map to FGLT_EHIP.
 *   - Calls on distinct streams with distinct workspaces may run concurrently.
 *
 * Integer ranges: n < 2^31 (int32 vertex ids); the largest degree must be
 * below 2^21 so that every count (at most d_max^3) fits in int64.
 */
#ifndef FGLT_H
#define FGLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FGLT_OK = 0,
    FGLT_EINVAL = -1,        /* bad argument (NULL pointer, negative size, n >= 2^31, ...) */
    FGLT_ENOTCANON = -2,     /* the CSR is not canonical (see fglt_raw)                    */
    FGLT_EWORKSPACE = -3,    /* ws_bytes below the size the workspace query returns        */
    FGLT_EOVERFLOW = -4,     /* a degree >= 2^21: counts could overflow int64              */
    FGLT_EHIP = -5,          /* the HIP runtime reported an error                          */
    FGLT_EUNSUPPORTED = -6   /* a graph outside what the chosen path supports              */
} fglt_status;

#define FGLT_NORBITS 16
#define FGLT_MAX_DEGREE ((int64_t)1 << 21)

/* fglt_raw flags */
#define FGLT_NET 1u          /* write net frequencies (Table II applied) instead of raw */
#define FGLT_TIMING 2u       /* time each launch segment with HIP events on `stream` (fills
                                fglt_stats.seg_ms; adds a final synchronization)         */
/* Sub-dictionary transforms (Section V; Table II's caption): bits 16..31 of
 * the flags hold the index set s of a sub-dictionary Sigma of Sigma_16 as a
 * mask (bit k = orbit k), which must contain orbits 0 and 1; 0 there means
 * all 16 orbits.  `out` is then [n][|s|], the orbits of s in ascending order:
 * raw frequencies, or with FGLT_NET the sub-dictionary's net frequencies
 * f_s = U16(s,s)^{-1} \hat f_s (the sub-matrix of Table II on s).  Where s
 * holds, with each orbit, every higher orbit its row of U16 reaches (as
 * {0..4} does), f_s equals those columns of the full net transform; other
 * sets give net frequencies relative to Sigma.  Only the passes that the
 * orbits of s need are run: the triangle pass for any of 4, 5, 6, 9, 10, 11,
 * 13, 14, 15; the clique/diamond pass for 13 or 15; the second row pass for
 * 5, 9, 10, 14 (or 13, 15); the 4-cycle pass (and its work lists) for 12. */
#define FGLT_SIGMA(mask) ((unsigned)((mask) & 0xffffu) << 16)
#define FGLT_SIGMA_MASK(flags) (((flags) >> 16) & 0xffffu)
#define FGLT_SIGMA5 FGLT_SIGMA(0x001fu)  /* Theorem 1: orbits 0-4, [n][5] */
#define FGLT_VALIDATE 16u    /* wait for the transform and return the device status word's
                                verdict (FGLT_ENOTCANON, FGLT_EOVERFLOW) instead of FGLT_OK */
#define FGLT_PROGRESS 32u    /* report each launch segment's end on stderr as the stream
                                reaches it (a host function enqueued on `stream`; the 4-cycle
                                window kernels report one by one): a line per step of a
                                transform that runs for minutes                            */
#define FGLT_WORKMODEL 8u    /* also count the work terms of the byte model (statistics only,
                                not part of the transform; needs `stats`): min_sum and
                                k4_merge of fglt_stats                                    */

/* Launch segments of fglt_raw, in execution order (indices into seg_ms). */
enum {
    FGLT_SEG_CHECK = 0,      /* input checks                                     */
    FGLT_SEG_RELABEL,        /* degree ranking, relabelled and re-sorted rows    */
    FGLT_SEG_STRUCTURE,      /* N-/N+ split, mirror positions, work counts, tiers */
    FGLT_SEG_TRI1_WAVE,      /* triangle pass (C3), wavefront tier                */
    FGLT_SEG_TRI1_LDS,       /* triangle pass, workgroup/LDS tier                 */
    FGLT_SEG_TRI1_GLOBAL,    /* triangle pass, hub tier and the chunked tier above */
    FGLT_SEG_FILL,           /* C3 mirrored to the lower entries, c3 by row sums,
                                row pass 1: A p1, A (p1-1)(p1-2)/2               */
    FGLT_SEG_TRI2_WAVE,      /* clique/diamond pass, wavefront tier               */
    FGLT_SEG_TRI2_LDS,       /* clique/diamond pass, LDS-bitmap tier              */
    FGLT_SEG_TRI2_GLOBAL,    /* clique/diamond pass, hub tier and the tier above it
                                with bitmaps in workspace slots                   */
    FGLT_SEG_L2,             /* row pass 2: A p2, A c3, C3 (p1-2), C(C3, 2), and the
                                clique/diamond counts stored per entry            */
    FGLT_SEG_C4_WAVE,        /* empty: the 4-cycle pass's wavefront, workgroup and
                                packed-hash tiers and the window tier's setup run on
                                a second stream beside the triangle segments       */
    FGLT_SEG_C4_BLOCK,       /* empty (as above)                                  */
    FGLT_SEG_C4_HASH,        /* empty: the window tier's per-entry table is built
                                on the second stream beside row pass 2            */
    FGLT_SEG_C4_WINDOW,      /* 4-cycle pass, dense-counter window tier (kernel)  */
    FGLT_SEG_FINALIZE,       /* Table I assembly, Table II, scatter to caller order */
    FGLT_NSEG
};

/*
 * Canonical adjacency from an edge list (the simple undirected graph of
 * Section I: symmetric 0/1 A, no self-loops, no multiple edges).
 *   n            number of vertices
 *   num_edges    number of input pairs
 *   src, dst     [num_edges] int32 endpoints, any order, may repeat, may be self-loops
 *   offsets      out [n+1] int64 row offsets
 *   indices      out, capacity 2*num_edges int32, rows strictly increasing
 *   nnz          out, device int64 scalar: the number of directed entries (2m);
 *                set to -1 if an endpoint lies outside [0, n) (offsets and
 *                indices are then undefined)
 *   ws, ws_bytes device workspace of at least fglt_build_csr_workspace(n, num_edges) bytes
 * Asynchronous; never synchronizes.
 */
size_t fglt_build_csr_workspace(int64_t n, int64_t num_edges);
int fglt_build_csr(int64_t n, int64_t num_edges, const int32_t* src, const int32_t* dst,
                   int64_t* offsets, int32_t* indices, int64_t* nnz,
                   void* ws, size_t ws_bytes, void* stream);

/* Statistics of the last fglt_raw call, filled when a host pointer is passed. */
typedef struct {
    int64_t n, nnz;              /* vertices, directed entries (2m)                       */
    int64_t d_max;               /* largest degree                                        */
    int64_t dplus_max;           /* largest out-degree under the degree ordering          */
    int64_t tri_items;           /* sum over oriented edges u->v of d+(v): merge work    */
    int64_t wedge_items;         /* rank-ordered wedges visited by the 4-cycle pass      */
    int64_t tri_tier_vertices[3]; /* vertices per triangle/clique tier: wave, LDS, global  */
    int64_t c4_tier_vertices[4];  /* vertices per 4-cycle tier: wave, block, hash, window  */
    int64_t tri_items_tier[3];    /* merge items per triangle/clique tier                  */
    int64_t wedge_items_tier[4];  /* wedges per 4-cycle tier                               */
    int64_t triangles;           /* triangles in the graph                                */
    int64_t min_sum;             /* with FGLT_WORKMODEL: sum over edges of min(d_i, d_j), the
                                    merge work of one oriented triangle listing (else 0)  */
    int64_t k4_merge;            /* with FGLT_WORKMODEL: sum over oriented triangles
                                    u < v < w of |N+(u) & N+(v)| + d+(w), the merge steps
                                    of an oriented 4-clique listing (else 0)              */
    float seg_ms[FGLT_NSEG];     /* with FGLT_TIMING: milliseconds per launch segment     */
} fglt_stats;

/* Tier thresholds of fglt_raw (host struct); 0 selects a default.  A vertex u
 * with out-degree D (under the degree ordering) is counted by one wavefront if
 * D <= tri_wave_max (<= 64), by a workgroup with LDS bitmaps if
 * D <= tri_lds_max (<= 512), by a 1024-thread workgroup with LDS position
 * map and bitmap rows in the workspace if D <= tri_hub_max (<= 1024), else
 * by chunks of its items spread over all workgroups (triangle pass) or a
 * 1024-thread workgroup with bitmaps in the workspace (clique pass).  The 4-cycle pass goes by the number W of rank-ordered wedges of
 * u: one wavefront if W <= c4_wave_max (<= 128), a workgroup with an LDS hash
 * if W <= c4_block_max (<= 2048), a large workgroup with a packed LDS hash if
 * W <= c4_hash_max (<= 16384) and the counts fit the packing, else dense LDS
 * counters over windows of ranks.  Any setting gives the same result; only
 * the speed changes. */
typedef struct {
    int32_t tri_wave_max;   /* default 64   */
    int32_t tri_lds_max;    /* default 512  */
    int32_t c4_wave_max;    /* default 128; -1 disables the tier */
    int32_t c4_block_max;   /* default 2048; -1 disables the tier */
    int32_t c4_hash_max;    /* default 16384; -1 disables the tier */
    int32_t c4_window_rows; /* window tier, how a middle's row is cut at the window
                               boundaries: 0 (default) a per-entry table where it fits the
                               workspace, else 1; 1 a per-vertex table; 2 binary searches */
    int32_t tri_hub_max;    /* out-degree up to which a vertex beyond the LDS tier is counted
                               by a 1024-thread workgroup with its position map (and, in the
                               clique pass, its adjacency bitmaps) in LDS; default 1024,
                               -1 disables the hub tier (every such vertex uses bitmaps in
                               the workspace) */
    int32_t c4_window_group; /* window tier, windows per job of a vertex with more than 1024
                               middles whose runs are searched (or, with 32-bit counters,
                               bracketed by the vertex table), each middle's run kept
                               between them: 0 (default) up to 16 as the tier's size allows,
                               k >= 1 exactly k (at most 1024) */
} fglt_raw_plan;

/*
 * Raw frequencies \hat f (Table I) of every vertex, or net frequencies
 * (Table I then Table II) with flags & FGLT_NET.
 *   n, nnz       vertices and directed entries of the CSR
 *   offsets      [n+1] int64, offsets[0] == 0, non-decreasing, offsets[n] == nnz
 *   indices      [nnz] int32; the CSR must be canonical: symmetric, no
 *                self-loops, no repeated entry in a row (rows need not be sorted)
 *   out          out [n][16] int64, or [n][|s|] with a sub-dictionary FGLT_SIGMA(s)
 *   ws, ws_bytes device workspace of at least fglt_raw_workspace(n, nnz) bytes
 *   flags        FGLT_NET, FGLT_TIMING, FGLT_VALIDATE, FGLT_WORKMODEL, FGLT_PROGRESS and a
 *                sub-dictionary FGLT_SIGMA(s), or 0; a mask without orbits 0
 *                and 1 is FGLT_EINVAL
 *   plan         (host) optional tier thresholds, NULL for the defaults
 *   stats        (host) optional, filled on success
 * The CSR is checked on the device (offsets, index range, self-loops,
 * repeated entries, symmetry, degrees below 2^21); a failed check sets the
 * workspace's status word and every later kernel that would index by the
 * input leaves at once (the output is then undefined).
 * Asynchronous: without FGLT_VALIDATE, FGLT_TIMING and `stats` it enqueues
 * every launch on `stream` (tier sizes and choices are read on the device)
 * and returns FGLT_OK without waiting, so it can be captured into a HIP graph;
 * fglt_raw_status() reads the status word afterwards.  With FGLT_VALIDATE or
 * `stats` it waits for the stream once, at the end, and returns
 * FGLT_ENOTCANON for a CSR that breaks the contract, FGLT_EOVERFLOW for a
 * degree >= 2^21.  FGLT_TIMING records events and is read at that wait.
 * With a sub-dictionary beyond {0..11} the transform also uses a second
 * stream of the calling thread, forked from and joined back into `stream`.
 */
size_t fglt_raw_workspace(int64_t n, int64_t nnz);
int fglt_raw(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices,
             int64_t* out, void* ws, size_t ws_bytes, unsigned flags, const fglt_raw_plan* plan,
             fglt_stats* stats, void* stream);
/* The status word of the last fglt_raw on this workspace (the same `ws`
 * pointer): FGLT_OK, FGLT_ENOTCANON or FGLT_EOVERFLOW.  Synchronizes with
 * `stream` (the stream that call used). */
int fglt_raw_status(const void* ws, void* stream);

/*
 * fglt_raw without a workspace argument, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: tight serving loops,
 * harnesses that forbid allocation).  The workspace is a device array of
 * FGLT_NOALLOC_SCRATCH_BYTES inside the library, one per device, held from
 * the library's load until the process ends; its device address is taken
 * with hipGetSymbolAddress on the first call on each device.  The call
 * itself allocates nothing (no hipMalloc, no stream or event creation; it
 * runs every kernel on `stream`).
 *   n, nnz, offsets, indices, out, flags, plan, stats   as for fglt_raw;
 *                FGLT_TIMING and FGLT_PROGRESS are not offered (FGLT_EINVAL); FGLT_VALIDATE is
 *                implied (the caller cannot reach the array's status word)
 * Returns FGLT_EWORKSPACE when fglt_raw_workspace(n, nnz) exceeds
 * FGLT_NOALLOC_SCRATCH_BYTES (1.2M to 1.6M directed entries fit).  Every call
 * on a device shares that device's array and overwrites it, so calls that
 * overlap on one device (different streams or threads) race: the caller
 * serializes them.  Waits for `stream` once, at the end (FGLT_VALIDATE).
 */
#define FGLT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int fglt_raw_noalloc(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices,
                     int64_t* out, unsigned flags, const fglt_raw_plan* plan, fglt_stats* stats, void* stream);

/*
 * Net from raw frequencies: f = U16^{-1} \hat f per vertex (Section V,
 * Table II), by exact integer back-substitution.  `net` may equal `raw`.
 * Asynchronous; never synchronizes.
 */
int fglt_net(int64_t n, const int64_t* raw, int64_t* net, void* stream);

/*
 * Graph-level totals (the relaxed, graph-level use of the encoding noted in
 * the Sigma_16 section): for each graph g and orbit k,
 *   totals[g][k] = (sum over the graph's vertices v of net[v][k]) / m_k,
 * where m_k is the number of vertices of orbit k's graphlet in orbit k
 * (Fig. 1; m = 1 2 2 1 3 2 2 3 1 1 2 1 4 2 2 4).  A net frequency counts the
 * induced copies of its graphlet at one vertex, so every orbit of a graphlet
 * gives that graphlet's number of induced copies in the graph.
 *   num_graphs   G >= 0 (< 2^31)
 *   vtx_offsets  [G+1] int64 on the device: graph g owns rows
 *                vtx_offsets[g] .. vtx_offsets[g+1]-1 of net (clamped to
 *                [0, n_total]); one graph: {0, n}
 *   net          [n_total][16] int64 on the device (fglt_net's or fglt_batch's output)
 *   totals       [G][16] int64 on the device, written
 * Asynchronous on `stream`.  FGLT_EINVAL for a negative size or a NULL pointer.
 */
int fglt_totals(int64_t num_graphs, const int64_t* vtx_offsets, int64_t n_total, const int64_t* net,
                int64_t* totals, void* stream);

/* Execution plan of fglt_batch (host struct); NULL or 0 fields select the
 * defaults.  Any plan gives the same result; only the speed changes.
 * fglt_batch_tune picks one for a given batch. */
typedef struct {
    int32_t threads;        /* threads per workgroup: 64, 128, 256, 512 or 1024 (default 256) */
    int32_t hub_degree;     /* vertices of at least this degree are taken by a whole wavefront in
                               the last pass, the others by one thread each (default and -1:
                               none) */
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit (256 of them) that take the
                               graphs, largest first, from a device work queue (default 64, at
                               most 64; never more workgroups than graphs) */
    int32_t use_graph;      /* 1: replay a captured hipGraph for this stream and shape (default 0) */
} fglt_batch_plan;

#define FGLT_BATCH_MAX_N 512

/*
 * Net frequencies of G independent graphs in one fused launch.
 *   num_graphs   G
 *   vtx_offsets  [G+1] int64: graph g owns vertices vtx_offsets[g] .. vtx_offsets[g+1]-1
 *   n_total      vtx_offsets[G]
 *   nnz_total    offsets[n_total]
 *   offsets      [n_total+1] int64 block-diagonal CSR (global vertex ids)
 *   indices      [nnz_total] int32, canonical as for fglt_raw; every entry of a
 *                row of graph g must lie in graph g's vertex range
 *   net          out [n_total][16] int64
 *   plan         (host) optional execution plan
 *   ws, ws_bytes device workspace of at least fglt_batch_workspace(...) bytes
 * Every graph must have at most FGLT_BATCH_MAX_N vertices (FGLT_EUNSUPPORTED
 * otherwise, checked on the host from the (host) copy `vtx_offsets_host`).
 * Entries that break the contract are skipped on the device and recorded in
 * a device status word, read by fglt_batch_status().  Asynchronous; never
 * synchronizes, so it can be captured into a HIP graph.
 */
size_t fglt_batch_workspace(int32_t num_graphs, int64_t n_total, int64_t nnz_total);
int fglt_batch(int32_t num_graphs, const int64_t* vtx_offsets, const int64_t* vtx_offsets_host,
               int64_t n_total, int64_t nnz_total, const int64_t* offsets, const int32_t* indices,
               int64_t* net, const fglt_batch_plan* plan, void* ws, size_t ws_bytes, void* stream);
/*
 * Autotuner of fglt_batch: times candidate plans on the caller's batch (the
 * same arguments as fglt_batch) and writes the fastest to *plan_out
 * (use_graph 0).  The candidates are threads 128, 256, 512 x hub_degree 16,
 * 32, 64, none x blocks_per_cu 2, 4, 8, 64; each runs once untimed, then `reps`
 * times (1..100) between HIP events on `stream`, and the median decides.  The
 * choice is cached inside the library by (G, n_total, nnz_total, the
 * histogram of graph sizes in 16 bins of 32 vertices): a later call with the
 * same key returns it at once without timing.  Writes `net` as fglt_batch
 * does.  Synchronizes with `stream`.  FGLT_EINVAL for bad arguments, else
 * fglt_batch's status.
 */
int fglt_batch_tune(int32_t num_graphs, const int64_t* vtx_offsets, const int64_t* vtx_offsets_host,
                    int64_t n_total, int64_t nnz_total, const int64_t* offsets, const int32_t* indices,
                    int64_t* net, void* ws, size_t ws_bytes, int32_t reps, fglt_batch_plan* plan_out,
                    void* stream);
/* Reads the status word of the last fglt_batch on this workspace (synchronizes
 * with `stream`): FGLT_OK or FGLT_ENOTCANON. */
int fglt_batch_status(const void* ws, void* stream);
/* Frees the HIP graphs cached for `stream` (NULL: all). */
int fglt_batch_release(void* stream);

const char* fglt_status_string(int status);
int fglt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FGLT_H */
