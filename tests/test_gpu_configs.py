"""Full-size workloads on the GPU against the oracle's stored digests.

tests/golden/digests.json holds, for each named workload, the sha256 of the
oracle's canonical CSR and of its n x 16 net array over every vertex, written
by tests/golden/make_digests.py (which calls only the oracle and the
generators).  The GPU path builds the CSR with fglt_build_csr and runs the
transform exactly as bench.py times it; both digests must match bit for bit.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests._util import ROOT, say, stratified_sample

pytestmark = pytest.mark.gpu

DIGESTS = os.path.join(ROOT, "tests", "golden", "digests.json")


def _digests():
    return json.load(open(DIGESTS)) if os.path.exists(DIGESTS) else {}


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def fg():
    import paper_2007_11111_amd as fg
    assert torch.cuda.is_available()
    return fg


def _edges(name):
    g = graphgen.make(name)
    if isinstance(g, list):
        src, dst, base = [], [], 0
        for x in g:
            src.append(x.src.astype(np.int64) + base)
            dst.append(x.dst.astype(np.int64) + base)
            base += x.n
        return base, np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)
    return g.n, g.src, g.dst


def _invariants(f, raw):
    S = f.sum(0)
    assert (f[:, 0] == 1).all()
    assert (f >= 0).all() and (raw >= f).all()
    assert S[2] == 2 * S[3] and S[5] == S[6] and S[7] == 3 * S[8]
    assert 2 * S[9] == S[10] and S[9] == S[11] and S[13] == S[14]
    assert S[4] % 3 == 0 and S[12] % 4 == 0 and S[15] % 4 == 0
    np.testing.assert_array_equal(f @ oracle.U16().T, raw)


@pytest.mark.parametrize("name", ["er", "batch", "rmat18", "cl", "rmat22"])
def test_workload_digest(fg, name):
    d = _digests().get(name)
    if d is None:
        pytest.skip(f"no stored oracle digest for {name}")
    n, src, dst = _edges(name)
    say(f"workload {name}: n={n} pairs={src.size}")
    off, idx = fg.build_csr(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    torch.cuda.synchronize()
    off_h, idx_h = off.cpu().numpy(), idx.cpu().numpy()
    assert sha(off_h, idx_h) == d["csr_sha256"], "fglt_build_csr differs from the oracle's canonical CSR"
    say(f"workload {name}: transform nnz={idx.numel()}")
    raw = fg.raw(off, idx)
    f = fg.net(raw)
    torch.cuda.synchronize()
    f_h = f.cpu().numpy()
    if sha(f_h) != d["net_sha256"]:
        colsum = f_h.sum(0).tolist()
        raise AssertionError(f"net digest mismatch; column sums {colsum} vs oracle {d['net_colsum']}")
    _invariants(f_h, raw.cpu().numpy())
    # the window tier's other row cuts (vertex table, binary searches) give the
    # same digest; R-MAT 22 (d_max >= 65536) runs them with 32-bit counters
    for rows in (1, 2):
        say(f"workload {name}: c4_window_rows={rows}")
        f2 = fg.net(fg.raw(off, idx, plan={"c4_window_rows": rows}))
        torch.cuda.synchronize()
        assert sha(f2.cpu().numpy()) == d["net_sha256"], f"net digest mismatch with c4_window_rows={rows}"
    # 16 windows per job of every many-middle vertex whatever the tier's size
    # (R-MAT 22's 23 vertices of degree >= 65536 keep one per window by
    # default): bracketed runs with the default row cuts, searched ones with 2
    for rows in (0, 2):
        say(f"workload {name}: c4_window_group=16 c4_window_rows={rows}")
        f2 = fg.net(fg.raw(off, idx, plan={"c4_window_rows": rows, "c4_window_group": 16}))
        torch.cuda.synchronize()
        assert sha(f2.cpu().numpy()) == d["net_sha256"], f"net digest mismatch with grouped windows, rows={rows}"
    # the transform with Sigma_5 gives the first five columns (raw and net)
    say(f"workload {name}: sigma5")
    s5n = fg.raw(off, idx, net=True, sigma5=True)
    s5r = fg.raw(off, idx, sigma5=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s5n.cpu().numpy(), f_h[:, :5])
    np.testing.assert_array_equal(s5r.cpu().numpy(), raw.cpu().numpy()[:, :5])
    # a stratified vertex sample recomputed live by the oracle (small degrees only:
    # the oracle's per-vertex cost grows with the square of the neighbourhood)
    deg = np.diff(off_h)
    sel = stratified_sample(deg, per_bin=40, top=0, seed=7, max_degree=64)
    say(f"workload {name}: live oracle sample of {sel.size}")
    np.testing.assert_array_equal(f_h[sel], oracle.net(off_h, idx_h, sel))


def _batch_union_on_device(fg, graphs):
    """The batch workload's block-diagonal CSR built on the device with
    fglt_build_csr from the union of the graphs' edge lists (no edge crosses
    two graphs), as bench.py builds it."""
    sizes = np.array([g.n for g in graphs], dtype=np.int64)
    vtx = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    base = np.repeat(vtx[:-1], [g.src.size for g in graphs])
    src = (np.concatenate([g.src for g in graphs]).astype(np.int64) + base).astype(np.int32)
    dst = (np.concatenate([g.dst for g in graphs]).astype(np.int64) + base).astype(np.int32)
    off, idx = fg.build_csr(int(vtx[-1]), torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    return torch.from_numpy(vtx), off, idx


@pytest.mark.parametrize("name", ["rmat18", "cl"])
def test_workload_digest_last_tier(fg, name):
    """Every vertex of out-degree above 1 in the last triangle and clique tiers
    (the chunked triangle kernel and the clique kernel with bitmaps in the
    workspace), against the oracle's digest.  With 10^6 vertices (Chung-Lu),
    N+(u) of most vertices spans more ranks than the LDS bitmap covers, so
    their positions come from the sampled search of the row."""
    d = _digests().get(name)
    if d is None:
        pytest.skip(f"no stored oracle digest for {name}")
    n, src, dst = _edges(name)
    off, idx = fg.build_csr(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    say(f"workload {name}: last tiers only")
    plan = {"tri_wave_max": 1, "tri_lds_max": 1, "tri_hub_max": -1}
    f = fg.net(fg.raw(off, idx, plan=plan))
    torch.cuda.synchronize()
    assert sha(f.cpu().numpy()) == d["net_sha256"], "net digest mismatch with the last tiers only"


def test_batch_workload_through_fglt_batch(fg):
    """The 4096-graph batch that bench.py times, through fglt_batch itself, one
    launch and by HIP-graph replay (three replays with eager work between
    them): every replay matches the oracle's stored net digest of the batch."""
    d = _digests().get("batch")
    if d is None:
        pytest.skip("no stored oracle digest for batch")
    graphs = graphgen.make("batch")
    vtx, off, idx = _batch_union_on_device(fg, graphs)
    torch.cuda.synchronize()
    assert sha(off.cpu().numpy(), idx.cpu().numpy()) == d["csr_sha256"]
    say(f"batch workload: G={len(graphs)} n={int(vtx[-1])} eager")
    out = fg.batch(vtx, off, idx)
    torch.cuda.synchronize()
    assert sha(out.cpu().numpy()) == d["net_sha256"]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(3):
            say(f"batch workload: graph replay {rep}")
            out2 = torch.full_like(out, -1)
            fg.batch(vtx, off, idx, out=out2, plan={"use_graph": 1}, stream=s)
            s.synchronize()
            assert sha(out2.cpu().numpy()) == d["net_sha256"], f"replay {rep}"
            _ = torch.ones(4096, device="cuda").cumsum(0).sum().item()  # eager work between replays
    fg.batch_release(s)


def _work_model_host(off, idx):
    """min_sum and the oriented 4-clique merge steps of a small canonical CSR
    by plain enumeration (degree order, ties by id)."""
    n = off.size - 1
    deg = np.diff(off)
    key = [(int(deg[v]), v) for v in range(n)]
    nplus = [set(int(w) for w in idx[off[v]:off[v + 1]] if key[int(w)] > key[v]) for v in range(n)]
    ms = ko = 0
    for u in range(n):
        for v in nplus[u]:
            ms += int(deg[u])
            T = nplus[u] & nplus[v]
            ko += len(T) * len(T) + sum(len(nplus[w]) for w in T)
    return ms, ko


def test_work_model_counts(fg):
    cases = [("er", graphgen.make("er")), ("cl3000", graphgen.chung_lu(3000, 2.3, 12.0, 400.0, seed=9)),
             ("K30", graphgen.clique(30)), ("star", graphgen.star(50))]
    for name, g in cases:
        o, i = oracle.canonical_csr(g.n, g.src, g.dst)
        say(f"work model {name}")
        _, st = fg.raw(torch.from_numpy(o).cuda(), torch.from_numpy(i).cuda(), stats=True, workmodel=True)
        ms, ko = _work_model_host(o, i)
        assert (st["min_sum"], st["k4_merge"]) == (ms, ko), name
    # the Erdos-Renyi workload's figures as the byte model states them
    o, i = oracle.canonical_csr(2000, graphgen.make("er").src, graphgen.make("er").dst)
    assert _work_model_host(o, i) == (94135, 502)
