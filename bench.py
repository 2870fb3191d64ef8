#!/usr/bin/env python3
"""Benchmark of the fast graphlet transform on one MI355X.

One step is one complete 16-orbit transform of the Chung-Lu workload
(n = 1,000,000, degree exponent 2.1, mean degree 20, cap 50,000): from the
canonical CSR resident in HBM to the n x 16 int64 net frequencies resident in
HBM (fglt_raw with the Table II conversion fused).  The CSR is built once,
before the timed region, with fglt_build_csr (its time is reported apart).

Prints one JSON line:
  value       undirected edges per second, m / (seconds per step)
  roofline    the dominant kernel segment: its algorithmic bytes per launch
              over its average duration, timed live with HIP events on the
              library's stream; traffic from committed rocprofv3 counters
  cpu_baseline  the CPU oracle timed on a bounded vertex sample of the same graph
  extra       per-segment times, the batched workload (4096 graphs, one launch)
              against a per-graph launch loop, and the CSR build time

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload cl|er|rmat22]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# Algorithmic bytes per unit of work of each counting segment (see the kernel
# notes in the sources): unit, bytes per unit.
SEG_UNITS = {
    "l2": ("entry", 36),         # row, index, C3, degree, p2 and c3 of the neighbour, clique counts
    "tri1_wave": ("item", 4),    # one out-list index per merge item
    "tri1_lds": ("item", 4),
    "tri1_global": ("item", 4),
    "tri2_wave": ("item", 8),    # out-list index + its C3 per merge item
    "tri2_lds": ("item", 8),
    "tri2_global": ("item", 8),
    "c4_wave": ("wedge", 8),     # wedge end read in the count and attribution passes
    "c4_block": ("wedge", 8),
    "c4_hash": ("wedge", 8),
    "c4_window": ("wedge", 8),
    "fill": ("entry", 16),       # row, index, mirror's C3, gathered degree
    "finalize": ("vertex", 232), # 13 accumulators + degree + id in, 128 B row out
}


def seg_units(seg, st):
    kind, _ = SEG_UNITS[seg]
    if kind == "entry":
        return st["nnz"]
    if kind == "vertex":
        return st["n"]
    tier = {"wave": 0, "lds": 1, "global": 2, "block": 1, "hash": 2, "window": 3}[seg.split("_")[1]]
    if kind == "item":
        return st["tri_items_tier"][tier]
    return st["wedge_items_tier"][tier]


# The kernel behind each timed segment whose traffic the counters give.
SEG_KERNEL = {
    "c4_window": "k_c4_window", "c4_hash": "k_c4_hashbig", "c4_block": "k_c4_hash<4, 4096>",
    "c4_wave": "k_c4_hash<1, 256>", "tri1_wave": "k_tri1_wave", "tri1_lds": "k_tri1_lds",
    "tri2_wave": "k_tri2s_wave", "l2": "k_l2", "fill": "k_fill_c3", "finalize": "k_finalize",
}


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_11111_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def load_traffic(seg):
    """HBM bytes per launch of the kernel behind `seg` from the committed
    rocprofv3 counters (profiles/traffic.json), or None if absent or taken on a
    different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or seg not in SEG_KERNEL:
        return None
    try:
        t = json.load(open(path))
    except Exception:
        return None
    if t.get("source_sha256") != source_hash():
        return None
    k = SEG_KERNEL[seg]
    hits = [v for name, v in t.get("kernels", {}).items() if name == k or name.startswith(k + "<")]
    return max(v["bytes_per_launch"] for v in hits) if hits else None


def _counter_means(db):
    """Per-kernel mean of each counter (KiB for FETCH_SIZE / WRITE_SIZE) over
    the dispatches of a rocprofv3 results database."""
    import collections
    import sqlite3
    con = sqlite3.connect(db)
    cur = con.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(counters_collection)")]
    ki, ci, vi = cols.index("kernel_name"), cols.index("counter_name"), cols.index("value")
    di = cols.index("dispatch_id")
    tot = collections.defaultdict(float)
    disp = collections.defaultdict(set)
    for r in cur.execute("select * from counters_collection"):
        name = r[ki].split("(")[0].replace("void ", "").replace("fglt::", "")
        tot[(name, r[ci])] += r[vi]
        disp[(name, r[ci])].add(r[di])
    return {k: v / len(disp[k]) for k, v in tot.items()}


def write_traffic(prof_dir, command):
    """profiles/traffic.json from four rocprofv3 --pmc runs under prof_dir
    (fetch/, write/: the benchmark; cfetch/, cwrite/: --copy-calibration 1024).
    Each counter is scaled by what it reads for the plain 1 GiB device copy."""
    import glob
    def db(sub):
        return glob.glob(os.path.join(prof_dir, sub, "*_results.db"))[0]
    copy_bytes = 1024 << 20
    cf = _counter_means(db("cfetch"))
    cw = _counter_means(db("cwrite"))
    fetch_copy = cf[("__amd_rocclr_copyBuffer", "FETCH_SIZE")] * 1024
    write_copy = cw[("__amd_rocclr_copyBuffer", "WRITE_SIZE")] * 1024
    fs, ws_ = copy_bytes / fetch_copy, copy_bytes / write_copy
    f = _counter_means(db("fetch"))
    w = _counter_means(db("write"))
    kernels = {}
    for (name, ctr), v in f.items():
        if ctr != "FETCH_SIZE" or not name.startswith("k_"):
            continue
        wr = w.get((name, "WRITE_SIZE"), 0.0)
        kernels[name] = {"fetch_kib": round(v, 1), "write_kib": round(wr, 1),
                         "bytes_per_launch": int(v * 1024 * fs + wr * 1024 * ws_)}
    out = {"source_sha256": source_hash(), "command": command,
           "calibration": {"copy_bytes": copy_bytes, "fetch_bytes_read": fetch_copy, "write_bytes_read": write_copy,
                           "fetch_scale": fs, "write_scale": ws_},
           "kernels": dict(sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"]))}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def cpu_baseline(off, idx, m, sample, seed=0):
    import oracle
    n = off.shape[0] - 1
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(n, size=min(sample, n), replace=False))
    t0 = time.perf_counter()
    oracle.net(off, idx, sel)
    dt = time.perf_counter() - t0
    frac = sel.size / n
    return {
        "value": m * frac / dt,
        "unit": "edges/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{sel.size} uniformly drawn vertices of {n} ({100 * frac:.1f}%), all 16 orbits, "
                  f"{dt:.1f} s; value = m * (sample/n) / seconds",
    }


def serving_leg(fg, torch, num=24, qps=100.0, seed=5):
    """Serving: Poisson arrivals (rate qps) of Chung-Lu requests with
    n = 10^U[3,6] through the HBM-budget server (GpuExecutor, four streams);
    latency from submission to result, after one warm-up request."""
    import graphgen
    from paper_2007_11111_amd.server import GpuExecutor, Server
    csrs = []
    for g in graphgen.serving_requests(num, seed):
        o, i = fg.build_csr(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda())
        csrs.append((o.cpu().numpy(), i.cpu().numpy()))
    arrivals = graphgen.poisson_arrivals(num, qps, seed)
    srv = Server(GpuExecutor(), budget_bytes=64 << 30, streams=4)
    lat = []
    try:
        srv.submit(*csrs[0]).result(timeout=300).release()
        futs = []
        t0 = time.perf_counter()
        for k, (o, i) in enumerate(csrs):
            wait = t0 + arrivals[k] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            ts = time.perf_counter()
            f = srv.submit(o, i)
            f.add_done_callback(lambda _f, ts=ts: lat.append(time.perf_counter() - ts))
            futs.append(f)
        for f in futs:
            f.result(timeout=300).release()
        wall = time.perf_counter() - t0
    finally:
        srv.close()
    lat_ms = 1e3 * np.array(lat)
    edges = sum(int(i.size) // 2 for _, i in csrs)
    return {"requests": num, "qps_offered": qps, "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 3), "max_ms": round(float(lat_ms.max()), 3),
            "mean_n": round(float(np.mean([o.size - 1 for o, _ in csrs])), 1), "edges": edges,
            "wall_s": round(wall, 3)}


def batch_leg(fg, torch, steps):
    import graphgen
    import oracle
    graphs = graphgen.make("batch")
    csrs = [oracle.canonical_csr(g.n, g.src, g.dst) for g in graphs]
    vtx, off, idx = fg.batch_pack(csrs)
    off_d, idx_d = off.cuda(), idx.cuda()
    out = torch.empty((int(vtx[-1]), 16), dtype=torch.int64, device="cuda")
    for _ in range(3):
        fg.batch(vtx, off_d, idx_d, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fg.batch(vtx, off_d, idx_d, out=out)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    # graph-level totals of every graph of the batch (fglt_totals)
    vtx_d = vtx.to("cuda", torch.int64)
    tot = fg.totals(out, vtx_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tot = fg.totals(out, vtx_d)
    torch.cuda.synchronize()
    t_tot = (time.perf_counter() - t0) / steps
    # reference point: one fglt_raw + net per graph, one stream, same device
    dev = [(torch.from_numpy(o).cuda(), torch.from_numpy(i).cuda()) for o, i in csrs]
    for o, i in dev[:16]:
        fg.raw(o, i, net=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for o, i in dev:
        fg.raw(o, i, net=True)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    G = len(graphs)
    return {"graphs": G, "n_total": int(vtx[-1]), "nnz_total": int(idx.numel()),
            "ms_per_batch": 1e3 * t_batch, "graphs_per_s": G / t_batch,
            "per_graph_loop_ms": 1e3 * t_loop, "per_graph_loop_graphs_per_s": G / t_loop,
            "speedup_vs_loop": t_loop / t_batch, "totals_ms": 1e3 * t_tot}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cl", choices=["cl", "er", "rmat22", "cl_small", "rmat18"])
    ap.add_argument("--cpu-sample", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sigma5", action="store_true", help="skip the Sigma_5 leg (keeps profiles to the full path)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="only write profiles/traffic.json from rocprofv3 counter runs under DIR and exit")
    ap.add_argument("--traffic-command", default="", help="the command recorded with --traffic-from")
    args = ap.parse_args()
    if args.traffic_from:
        out = write_traffic(args.traffic_from, args.traffic_command)
        print(json.dumps(out["calibration"]))
        return
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the transform is not "
              "sharded across GPUs in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen
    import paper_2007_11111_amd as fg

    g = graphgen.make(args.workload)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off, idx = fg.build_csr(g.n, src, dst)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t0)
    n, nnz = g.n, int(idx.numel())
    m = nnz // 2
    out = torch.empty((n, 16), dtype=torch.int64, device="cuda")
    ws = torch.empty(fg.raw_workspace_bytes(n, nnz), dtype=torch.uint8, device="cuda")

    for _ in range(args.warmup):
        fg.raw(off, idx, net=True, out=out, workspace=ws)
    torch.cuda.synchronize()
    seg_sum = {}
    st = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = fg.raw(off, idx, net=True, out=out, workspace=ws, stats=True, timing=True)
        for k, v in st["seg_ms"].items():
            seg_sum[k] = seg_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    seg_avg = {k: v / args.steps for k, v in seg_sum.items()}
    # graph-level totals of the workload (fglt_totals on the net frequencies), after the timed steps
    fg.totals(out)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        fg.totals(out)
    torch.cuda.synchronize()
    totals_ms = 1e3 * (time.perf_counter() - t2) / args.steps
    # the transform with the sub-dictionary Sigma_5 (orbits 0-4) of the same graph
    sigma5_ms = None
    if not args.no_sigma5:
        out5 = torch.empty((n, 5), dtype=torch.int64, device="cuda")
        fg.raw(off, idx, net=True, out=out5, workspace=ws, sigma5=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(args.steps):
            fg.raw(off, idx, net=True, out=out5, workspace=ws, sigma5=True)
        torch.cuda.synchronize()
        sigma5_ms = 1e3 * (time.perf_counter() - t3) / args.steps
        del out5

    # dominant counting segment and its roofline
    counted = {k: v for k, v in seg_avg.items() if k in SEG_UNITS}
    dom = max(counted, key=counted.get)
    units = seg_units(dom, st)
    alg_bytes = units * SEG_UNITS[dom][1]
    dur_s = seg_avg[dom] / 1e3
    achieved = alg_bytes / dur_s / 1e9 if dur_s > 0 else 0.0
    path_bytes = sum(seg_units(k, st) * SEG_UNITS[k][1] for k in SEG_UNITS)
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": load_traffic(dom),
                "kernel": dom, "kernel_ms": round(seg_avg[dom], 4),
                "alg_bytes_per_launch": int(alg_bytes), "units_per_launch": int(units),
                "unit_of_work": SEG_UNITS[dom][0], "bytes_per_unit": SEG_UNITS[dom][1]}

    extra = {"build_csr_ms": round(build_ms, 3), "totals_ms": round(totals_ms, 4),
             "sigma5_ms": round(sigma5_ms, 4) if sigma5_ms else None,
             "sigma5_edges_per_s": round(m / (sigma5_ms / 1e3), 1) if sigma5_ms else None, "seg_ms": {k: round(v, 4) for k, v in seg_avg.items()},
             "path_alg_gbps": round(path_bytes / (ms_per_step / 1e3) / 1e9, 2),
             "stats": {k: v for k, v in st.items() if k != "seg_ms"}}
    if not args.no_batch:
        extra["batch"] = batch_leg(fg, torch, steps=max(3, args.steps))
    if not args.no_serving:
        extra["serving"] = serving_leg(fg, torch)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu = cpu_baseline(off.cpu().numpy(), idx.cpu().numpy(), m, args.cpu_sample)

    rec = {
        "metric": "edges/s, 16-orbit fast graphlet transform (raw + net), one graph",
        "value": m / (ms_per_step / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": {"cl": "chung_lu_n1M_exp2.1_mean20_cap50k", "er": "erdos_renyi_n2000_p0.005",
                                "rmat22": "rmat_scale22_ef16", "cl_small": "chung_lu_n100k",
                                "rmat18": "rmat_scale18_ef16"}[args.workload],
                   "n": n, "m": m, "d_max": st["d_max"], "seed": {"cl": 2, "er": 1, "rmat22": 3}.get(args.workload, 0),
                   "parallelism": "single-gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
