"""The Friendster-scale single-GPU run (Section VI's largest graph: 66M
vertices, 1.8B links), on a synthetic stand-in: R-MAT scale 26, edge factor
27 (0.57, 0.19, 0.19, 0.05), ids permuted -- 1.8e9 pairs on 67M vertices.

Opt-in (minutes of generation and oracle work): FGLT_FRIENDSTER_SCALE=S runs
the chunked R-MAT recipe at scale S (26 for the full size; smaller scales are
the steps up to it), and FGLT_FRIENDSTER_SIGMAS lists the sub-dictionary masks
to run (default 0x1f, Theorem 1's Sigma_5).  For each mask: fglt_build_csr on
the device against the oracle's canonical CSR (C route, every entry), the
transform timed with HIP events (one call, with per-segment events),
whole-graph invariants of the net counts, and
a degree-stratified vertex sample recomputed by the oracle (vertices whose
two-hop oracle cost stays bounded).  FGLT_FRIENDSTER_OUT names a JSON file for
the measured figures.  FGLT_FRIENDSTER_WS_EXTRA_GB gives the transform that
many GiB of workspace beyond fglt_raw_workspace's minimum (default 0): the
library keeps the triangle pass's neighbourhood bitmaps there for the clique
pass when all of them fit, instead of forming them again.
"""
import json
import os
import time

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests._util import say, stratified_sample

SCALE = os.environ.get("FGLT_FRIENDSTER_SCALE")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not SCALE, reason="opt-in: set FGLT_FRIENDSTER_SCALE (26 for the full size)")]


@pytest.fixture(scope="module")
def fg():
    import paper_2007_11111_amd as fg
    assert torch.cuda.is_available()
    return fg


def _cost_bounded_sample(off, idx, deg, budget, total_budget, seed):
    """Up to 24 vertices per log2-degree bin (degree <= 4096) whose oracle
    cost, the sum over v and its neighbours j of sum_{k in N(j)} d_k, is at
    most `budget`, taken in id order while their costs stay within `total_budget`."""
    cand = stratified_sample(deg, per_bin=24, top=0, seed=seed, max_degree=4096)
    keep, spent = [], 0
    for v in cand:
        js = np.concatenate([[v], idx[off[v]:off[v + 1]]])
        cost = 0
        for jj in js:
            cost += int(deg[idx[off[jj]:off[jj + 1]]].sum())
            if cost > budget:
                break
        if cost <= budget and spent + cost <= total_budget:
            keep.append(int(v))
            spent += cost
    return np.array(keep, dtype=np.int64)


def test_friendster_scale_sigma(fg):
    scale = int(SCALE)
    masks = [int(x, 0) for x in os.environ.get("FGLT_FRIENDSTER_SIGMAS", "0x1f").split(",")]
    name = f"rmat{scale}c"
    say(f"friendster-scale: generating {name}")
    t = time.perf_counter()
    g = graphgen.make(name)
    gen_s = time.perf_counter() - t
    say(f"friendster-scale: n={g.n} pairs={g.src.size} generated in {gen_s:.1f} s; device CSR")
    src, dst = torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    off, idx = fg.build_csr(g.n, src, dst)
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - t)
    del src, dst
    torch.cuda.empty_cache()
    say(f"friendster-scale: device CSR nnz={idx.numel()} in {build_ms:.1f} ms; oracle CSR")
    t = time.perf_counter()
    off_o, idx_o = oracle.canonical_csr_large(g.n, g.src, g.dst)
    ocsr_s = time.perf_counter() - t
    n = g.n
    del g
    np.testing.assert_array_equal(off.cpu().numpy(), off_o)
    np.testing.assert_array_equal(idx.cpu().numpy(), idx_o)
    deg = np.diff(off_o)
    say(f"friendster-scale: CSR equal (oracle {ocsr_s:.1f} s); d_max={deg.max()}")
    assert deg.max() < 2 ** 21
    sel = _cost_bounded_sample(off_o, idx_o, deg, budget=200_000_000, total_budget=20_000_000_000, seed=11)
    say(f"friendster-scale: oracle sample of {sel.size} vertices")
    t = time.perf_counter()
    raw_o = oracle.raw(off_o, idx_o, sel)
    oracle_s = time.perf_counter() - t
    say(f"friendster-scale: oracle sample in {oracle_s:.1f} s")
    nnz = int(idx.numel())
    extra = int(float(os.environ.get("FGLT_FRIENDSTER_WS_EXTRA_GB", "0")) * 2 ** 30)
    ws = torch.empty(fg.raw_workspace_bytes(n, nnz) + extra, dtype=torch.uint8, device="cuda")
    report = {"workload": f"rmat_scale{scale}_ef27_abcd0.57-0.19-0.19-0.05_permuted_chunked", "n": n,
              "m": nnz // 2, "d_max": int(deg.max()), "isolated": int((deg == 0).sum()),
              "generate_s": round(gen_s, 1), "build_csr_ms": round(build_ms, 1),
              "oracle_csr_s": round(ocsr_s, 1), "oracle_sample": int(sel.size),
              "oracle_sample_s": round(oracle_s, 1), "workspace_bytes": int(ws.numel()), "sigmas": {}}
    for mask in masks:
        cols = oracle.subdict_columns(mask)
        out = torch.empty((n, len(cols)), dtype=torch.int64, device="cuda")
        say(f"friendster-scale: transform sigma={hex(mask)}")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, st = fg.raw(off, idx, net=True, out=out, workspace=ws, sigma=mask, stats=True, timing=True,
                       progress=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        assert fg.raw_status(ws) == 0
        f = out.cpu().numpy()
        say(f"friendster-scale: sigma={hex(mask)} {ms:.1f} ms; segments "
            + json.dumps({k: round(v, 1) for k, v in st["seg_ms"].items() if v >= 0.05}))
        say(f"friendster-scale: tiers tri {list(st['tri_tier_vertices'])} c4 {list(st['c4_tier_vertices'])}; checks")
        # the oracle's sample, through the same sub-dictionary
        np.testing.assert_array_equal(f[sel], oracle.subdict(raw_o, mask))
        # whole-graph invariants of the net counts that every run has; a
        # column is an induced count (so never negative) when its row of
        # U16^-1 stays inside s
        S = f.sum(0)
        c = {k: i for i, k in enumerate(cols)}
        uinv = np.rint(np.linalg.inv(oracle.U16().astype(np.float64))).astype(np.int64)
        closed = [c[k] for k in cols if set(np.nonzero(uinv[k])[0]) <= set(cols)]
        assert (f[:, c[0]] == 1).all() and (f[:, closed] >= 0).all()
        np.testing.assert_array_equal(f[:, c[1]], deg)
        if 2 in c and 3 in c:
            assert S[c[2]] == 2 * S[c[3]]
        if 4 in c:
            assert S[c[4]] % 3 == 0
        report["sigmas"][hex(mask)] = {"ms": round(ms, 1), "edges_per_s": round((nnz // 2) / (ms / 1e3), 1),
                                       "seg_ms": {k: round(v, 2) for k, v in st["seg_ms"].items()},
                                       "tri_tier_vertices": st["tri_tier_vertices"],
                                       "c4_tier_vertices": st["c4_tier_vertices"],
                                       "column_sums": [int(x) for x in S]}
        del out
    path = os.environ.get("FGLT_FRIENDSTER_OUT")
    if path:
        with open(path, "w") as fh:
            json.dump(report, fh, indent=1)
    say(json.dumps(report))
