// api.hip -- C ABI entry points of the single-graph transform (fglt_raw,
// fglt_net) and the status helpers.  See include/fglt.h.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <initializer_list>

#include "raw.h"

using namespace fglt;

const char* const fglt::kSegNames[FGLT_NSEG] = {
    "check", "relabel", "structure", "tri1_wave", "tri1_lds", "tri1_global", "fill", "tri2_wave",
    "tri2_lds", "tri2_global", "l2", "c4_wave", "c4_block", "c4_hash", "c4_window", "finalize"};

// Runs on the runtime's callback thread when the stream reaches it; makes no HIP call.
void fglt::progress_line(void* what) {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    const double sec = std::chrono::duration<double>(clk::now() - t0).count();
    std::fprintf(stderr, "fglt: %s done (%.1f s)\n", static_cast<const char*>(what), sec);
    std::fflush(stderr);
}

namespace {

int status_from_err(u32 err) {
    if (err & ERR_DEGREE) return FGLT_EOVERFLOW;
    if (err) return FGLT_ENOTCANON;
    return FGLT_OK;
}

// A second stream of the calling thread on the current device (default
// priority) with a fork and a join event, created on first use and kept for
// the thread's lifetime.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, mid = nullptr, join = nullptr;
};

static hipError_t aux_stream(AuxStream*& out) {
    static constexpr int MAXDEV = 64;
    thread_local AuxStream aux[MAXDEV];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    AuxStream& a = aux[dev];
    if (!a.s) {
        if ((e = hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.mid, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) return e;
    }
    out = &a;
    return hipSuccess;
}

// The passes that the orbits of a sub-dictionary need (Table I): the
// triangle pass for any orbit that reads C3 or c3, the clique/diamond pass
// for the diamond off-cord and 4-clique orbits, row pass 2 for the sums over
// neighbours of p2, c3 and C3 (and the clique pass's per-entry counts, which
// it sums), the 4-cycle pass for the 4-cycle orbit.  Degrees, p2 and
// A C(p1-1, 2) (row pass 1) always run.
struct SubPasses {
    bool tri, clique, l2, c4;
};
static SubPasses sub_passes(unsigned s) {
    auto any = [s](std::initializer_list<int> ks) {
        for (int k : ks)
            if ((s >> k) & 1u) return true;
        return false;
    };
    SubPasses p;
    p.c4 = any({12});
    p.clique = any({13, 15});
    p.l2 = p.clique || any({5, 9, 10, 14});
    p.tri = p.l2 || any({4, 6, 11});
    return p;
}


// The last timing event; with statistics or FGLT_VALIDATE the one wait for
// the stream: the device plan (status word, tier sizes, work totals) and, with
// FGLT_TIMING, the segment times.  Without either, nothing is waited for and
// the status stays on the device (fglt_raw_status).
int finish(int64_t n, int64_t nnz, RawWs& w, SegTimer& tm, unsigned flags, fglt_stats* stats, hipStream_t s) {
    if (tm.on) FGLT_HIP_TRY(hipEventRecord(tm.ev[FGLT_NSEG], s));
    if (tm.last >= 0) tm.note(kSegNames[tm.last], s);
    if (!stats && !(flags & FGLT_VALIDATE)) return FGLT_OK;
    if (stats) {
        FGLT_HIP_TRY(launch_count_triangles(n, w, s));
        if (flags & FGLT_WORKMODEL) FGLT_HIP_TRY(launch_work_model(nnz, w, s));
    }
    DevPlan fin{};
    i64 g_total = 0;
    if (hipMemcpyAsync(&fin, w.plan, sizeof(DevPlan), hipMemcpyDeviceToHost, s) != hipSuccess) return FGLT_EHIP;
    if (stats && hipMemcpyAsync(&g_total, w.G + nnz, sizeof(i64), hipMemcpyDeviceToHost, s) != hipSuccess)
        return FGLT_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return FGLT_EHIP;
    const int st = status_from_err(fin.err);
    if (st) return st;
    if (stats) {
        stats->d_max = fin.d_max;
        stats->dplus_max = fin.dplus_max;
        stats->tri_items = g_total - fin.wedge_items;
        stats->wedge_items = fin.wedge_items;
        for (int k = 0; k < 3; ++k) {
            stats->tri_tier_vertices[k] = fin.n_tri[k];
            stats->tri_items_tier[k] = fin.tri_items_tier[k];
        }
        for (int k = 0; k < 4; ++k) {
            stats->c4_tier_vertices[k] = fin.n_c4[k];
            stats->wedge_items_tier[k] = fin.wedge_items_tier[k];
        }
        stats->triangles = fin.triangles / 6;  // twice at each of its three vertices
        stats->min_sum = fin.min_sum;
        stats->k4_merge = fin.k4_merge;
        if (tm.on) {
            for (int k = 0; k < FGLT_NSEG; ++k) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, tm.ev[k], tm.ev[k + 1]) != hipSuccess) return FGLT_EHIP;
                stats->seg_ms[k] = ms;
            }
        }
    }
    return FGLT_OK;
}

}  // namespace

extern "C" size_t fglt_raw_workspace(int64_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    Carver c(nullptr, 0);
    carve_raw(c, n, nnz);
    return c.used;
}

int fglt::raw_run(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices, int64_t* out, void* ws,
                  size_t ws_bytes, unsigned flags, const fglt_raw_plan* plan, fglt_stats* stats, void* stream,
                  bool one_stream) {
    if (n < 0 || n >= ((int64_t)1 << 31) || nnz < 0 || nnz >= ((int64_t)1 << 40)) return FGLT_EINVAL;
    if (n > 0 && (!offsets || !out || !ws)) return FGLT_EINVAL;
    if (nnz > 0 && !indices) return FGLT_EINVAL;
    if (flags & ~(FGLT_NET | FGLT_TIMING | FGLT_WORKMODEL | FGLT_VALIDATE | FGLT_PROGRESS | FGLT_SIGMA(0xffffu)))
        return FGLT_EINVAL;
    // the sub-dictionary (Section V): every orbit by default; {0, 1} in any subset
    const unsigned smask = FGLT_SIGMA_MASK(flags) ? FGLT_SIGMA_MASK(flags) : 0xffffu;
    if ((smask & 3u) != 3u) return FGLT_EINVAL;
    const SubPasses sp = sub_passes(smask);
    if (stats) {
        *stats = fglt_stats{};
        stats->n = n;
        stats->nnz = nnz;
    }
    if (n == 0) return nnz == 0 ? FGLT_OK : FGLT_ENOTCANON;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws, ws_bytes);
    RawWs w = carve_raw(c, n, nnz);
    if (!c.ok()) return FGLT_EWORKSPACE;

    SegTimer tm;
    struct EvGuard {
        SegTimer& t;
        ~EvGuard() {
            for (auto& e : t.ev)
                if (e) (void)hipEventDestroy(e);
        }
    } guard{tm};
    if (flags & FGLT_TIMING) {
        for (auto& e : tm.ev) FGLT_HIP_TRY(hipEventCreate(&e));
        tm.on = true;
    }
    tm.progress = (flags & FGLT_PROGRESS) != 0;

    // 1. input checks into the device status word; every later kernel that
    // indexes by the input's values leaves at once if a check failed
    tm.mark(FGLT_SEG_CHECK, s);
    FGLT_HIP_TRY(launch_check_input(n, nnz, offsets, indices, w, s));

    // 2. degree ranking, relabelled CSR, work counts, tiers, and the decisions
    // that depend on them, all on the device
    tm.mark(FGLT_SEG_RELABEL, s);
    FGLT_HIP_TRY(launch_rank_and_relabel(n, nnz, offsets, indices, w, s));
    tm.mark(FGLT_SEG_STRUCTURE, s);
    const Tiers tiers = tiers_from_plan(plan, n);
    FGLT_HIP_TRY(launch_structure(n, nnz, w, tiers, sp.c4, sp.clique, tiers.c4_rows, s));

    // 3. counting
    FGLT_HIP_TRY(fill_u32(w.acc, 2 * 10 * n, 0u, s));
    if (nnz > 0) FGLT_HIP_TRY(fill_u32(w.C3, nnz, 0u, s));
    const bool net = (flags & FGLT_NET) != 0;
    // the 4-cycle pass's hash tiers and window setup share no memory with the
    // triangle and clique passes: a second stream runs them alongside, and the
    // window kernels (after the join) take the whole GPU.  A sub-dictionary
    // runs only the passes its orbits need.
    AuxStream* aux = nullptr;
    hipStream_t s4 = s;
    if (sp.c4 && !one_stream) {
        FGLT_HIP_TRY(aux_stream(aux));
        FGLT_HIP_TRY(hipEventRecord(aux->fork, s));
        FGLT_HIP_TRY(hipStreamWaitEvent(aux->s, aux->fork, 0));
        s4 = aux->s;
    }
    if (sp.c4) FGLT_HIP_TRY(launch_c4_early(n, nnz, w, tiers.c4_rows, tiers.c4_group, s4));
    if (sp.tri) FGLT_HIP_TRY(launch_tri(n, nnz, w, 1, tiers.tri_hub, s, tm));
    else
        for (int seg = FGLT_SEG_TRI1_WAVE; seg <= FGLT_SEG_TRI1_GLOBAL; ++seg) tm.mark(seg, s);
    tm.mark(FGLT_SEG_FILL, s);
    FGLT_HIP_TRY(launch_fill_c3(nnz, w, s));
    if (sp.clique) FGLT_HIP_TRY(launch_tri(n, nnz, w, 2, tiers.tri_hub, s, tm));
    else
        for (int seg = FGLT_SEG_TRI2_WAVE; seg <= FGLT_SEG_TRI2_GLOBAL; ++seg) tm.mark(seg, s);
    // the bitmaps are dead now: the window tier's per-entry table goes there,
    // on the second stream beside row pass 2
    if (aux) {
        FGLT_HIP_TRY(hipEventRecord(aux->mid, s));
        FGLT_HIP_TRY(hipStreamWaitEvent(aux->s, aux->mid, 0));
    }
    if (sp.c4) FGLT_HIP_TRY(launch_c4_etab(n, nnz, w, tiers.c4_rows, tiers.c4_group, s4));
    if (aux) FGLT_HIP_TRY(hipEventRecord(aux->join, s4));
    tm.mark(FGLT_SEG_L2, s);
    if (sp.l2) FGLT_HIP_TRY(launch_l2(n, nnz, w, s));
    if (aux) FGLT_HIP_TRY(hipStreamWaitEvent(s, aux->join, 0));
    if (sp.c4) FGLT_HIP_TRY(launch_c4_late(n, nnz, w, tiers.c4_rows, tiers.c4_group, s, tm));
    else
        for (int seg = FGLT_SEG_C4_WAVE; seg <= FGLT_SEG_C4_WINDOW; ++seg) tm.mark(seg, s);
    tm.mark(FGLT_SEG_FINALIZE, s);
    if (smask == 0xffffu) FGLT_HIP_TRY(launch_finalize(n, w, out, net, s));
    else FGLT_HIP_TRY(launch_finalize_sub(n, w, out, net, smask, s));
    return finish(n, nnz, w, tm, flags, stats, s);
}

extern "C" int fglt_raw(int64_t n, int64_t nnz, const int64_t* offsets, const int32_t* indices, int64_t* out,
                        void* ws, size_t ws_bytes, unsigned flags, const fglt_raw_plan* plan, fglt_stats* stats,
                        void* stream) {
    return raw_run(n, nnz, offsets, indices, out, ws, ws_bytes, flags, plan, stats, stream, false);
}

extern "C" int fglt_raw_status(const void* ws, void* stream) {
    if (!ws) return FGLT_EINVAL;
    // the device plan is the workspace's first piece, at its first 256-byte boundary
    const uintptr_t a = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
    u32 err = 0;
    FGLT_HIP_TRY(hipMemcpyAsync(&err, (const void*)a, sizeof(u32), hipMemcpyDeviceToHost, (hipStream_t)stream));
    FGLT_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    return status_from_err(err);
}

extern "C" int fglt_net(int64_t n, const int64_t* raw, int64_t* net, void* stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return FGLT_EINVAL;
    if (n == 0) return FGLT_OK;
    if (!raw || !net) return FGLT_EINVAL;
    FGLT_HIP_TRY(launch_net(n, raw, net, (hipStream_t)stream));
    return FGLT_OK;
}

extern "C" const char* fglt_status_string(int status) {
    switch (status) {
        case FGLT_OK: return "ok";
        case FGLT_EINVAL: return "invalid argument";
        case FGLT_ENOTCANON: return "CSR is not canonical (symmetric, no self-loops, no repeated entries)";
        case FGLT_EWORKSPACE: return "workspace too small";
        case FGLT_EOVERFLOW: return "a degree is >= 2^21; counts could overflow int64";
        case FGLT_EHIP: return "HIP runtime error";
        case FGLT_EUNSUPPORTED: return "unsupported input for this path";
        default: return "unknown status";
    }
}

extern "C" int fglt_version(void) { return 1; }
