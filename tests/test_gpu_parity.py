"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Every comparison is exact int64 equality.  Tier plans force every vertex
through each kernel tier on small graphs, so each tier is checked against the
oracle, not only the tiers a graph would pick by itself.
"""
import math
import re

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests._util import csr_arrays, say

pytestmark = pytest.mark.gpu

C = math.comb

# Tier plans: default; everything in the wave tiers where allowed; everything
# in the LDS/workgroup tiers; the 4-cycle pass in the packed-hash tier where
# it fits; the triangle and clique passes in the hub tier (position map in
# LDS, bitmap rows in the workspace) and the 4-cycle pass in the window tier;
# the same with the hub tier off (bitmaps in the workspace).
PLANS = {
    "default": None,
    "wave": {"tri_wave_max": 64, "tri_lds_max": 64, "c4_wave_max": 128, "c4_block_max": 128, "c4_hash_max": 128},
    "block": {"tri_wave_max": 1, "tri_lds_max": 512, "c4_wave_max": -1, "c4_block_max": 2048, "c4_hash_max": -1},
    "hash": {"tri_wave_max": 1, "tri_lds_max": 512, "c4_wave_max": -1, "c4_block_max": -1, "c4_hash_max": 16384},
    "global": {"tri_wave_max": 1, "tri_lds_max": 1, "c4_wave_max": -1, "c4_block_max": -1, "c4_hash_max": -1},
    "nohub": {"tri_wave_max": 1, "tri_lds_max": 1, "tri_hub_max": -1, "c4_wave_max": -1, "c4_block_max": -1,
              "c4_hash_max": -1},
}


@pytest.fixture(scope="module")
def fg():
    import paper_2007_11111_amd as fg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fg._lib.lib()
    return fg


def to_dev(off, idx):
    return (torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda())


def gpu_raw(fg, off, idx, plan=None, net=False):
    o, i = to_dev(off, idx)
    out = fg.raw(o, i, net=net, plan=plan)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# ------------------------------------------------------------------ CSR build

@pytest.mark.parametrize("case", ["empty", "one", "loops_dups", "er", "cl"])
def test_build_csr_matches_oracle(fg, case):
    rng = np.random.default_rng(5)
    if case == "empty":
        n, src, dst = 0, np.zeros(0, np.int32), np.zeros(0, np.int32)
    elif case == "one":
        n, src, dst = 1, np.zeros(3, np.int32), np.zeros(3, np.int32)
    elif case == "loops_dups":
        n = 50
        src = rng.integers(0, n, 3000).astype(np.int32)
        dst = rng.integers(0, n, 3000).astype(np.int32)
    elif case == "er":
        g = graphgen.erdos_renyi(2000, 0.005, seed=1)
        n, src, dst = g.n, g.src, g.dst
    else:
        g = graphgen.chung_lu(60_000, 2.1, 20.0, 3000.0, seed=2)
        n, src, dst = g.n, g.src, g.dst
    say(f"build_csr case={case} n={n} pairs={src.size}")
    off_e, idx_e = oracle.canonical_csr(n, src, dst)
    o, i = fg.build_csr(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o.cpu().numpy(), off_e)
    np.testing.assert_array_equal(i.cpu().numpy(), idx_e)


def test_build_csr_rejects_out_of_range(fg):
    src = torch.tensor([0, 1, 7], dtype=torch.int32).cuda()
    dst = torch.tensor([1, 2, 0], dtype=torch.int32).cuda()
    with pytest.raises(fg.FgltError):
        fg.build_csr(5, src, dst)


# ------------------------------------------------------------------ worked example

@pytest.mark.parametrize("plan", list(PLANS))
def test_fig2(fg, fig2, plan):
    say(f"fig2 plan={plan}")
    off, idx = csr_arrays(fig2["n"], fig2["edges"])
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan]), fig2["raw"])
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan], net=True), fig2["net"])


# ------------------------------------------------------------------ small random graphs, every tier

def _small_graphs():
    rng = np.random.default_rng(2024)
    out = [(1, []), (2, [(0, 1)]), (7, []), (6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])]
    for _ in range(30):
        n = int(rng.integers(3, 60))
        p = float(rng.choice([0.05, 0.1, 0.3, 0.6, 0.9]))
        out.append((n, [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]))
    return out


@pytest.mark.parametrize("plan", list(PLANS))
def test_small_random_all_tiers(fg, plan):
    for gi, (n, edges) in enumerate(_small_graphs()):
        say(f"small graph {gi} n={n} m={len(edges)} plan={plan}")
        off, idx = csr_arrays(n, edges)
        exp = oracle.raw(off, idx)
        got = gpu_raw(fg, off, idx, PLANS[plan])
        np.testing.assert_array_equal(got, exp, err_msg=f"graph {gi}")
        np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan], net=True), oracle.raw_to_net(exp))


# ------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [2, 3, 4, 5, 30, 70, 600, 1070, 1100, 4200])
def test_clique(fg, n):
    """K_n: out-degree n-1 of the lowest vertex (600 reaches the hub tier,
    1070 its second round of out-neighbours per thread, 1100 the
    global-bitmap tier beyond it, 4200 the clique launch for out-degrees
    above 4096, and the top vertex's (n-1)(n-2) wedges the heavy 4-cycle
    tier)."""
    g = graphgen.clique(n)
    say(f"clique n={n}")
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = gpu_raw(fg, off, idx, net=True)
    exp = np.zeros(16, dtype=np.int64)
    exp[0], exp[1], exp[4], exp[15] = 1, n - 1, C(n - 1, 2), C(n - 1, 3)
    np.testing.assert_array_equal(f, np.tile(exp, (n, 1)))
    r = gpu_raw(fg, off, idx)
    a, b, c = n - 1, max(n - 2, 0), max(n - 3, 0)
    exp_raw = [1, a, a * b, C(a, 2), C(a, 2), a * b * c, a * b * c, a * C(b, 2), C(a, 3),
               c * C(a, 2), a * b * c, c * C(a, 2), a * C(b, 2), c * C(a, 2), a * C(b, 2), C(a, 3)]
    np.testing.assert_array_equal(r, np.tile(np.array(exp_raw, dtype=np.int64), (n, 1)))


@pytest.mark.parametrize("k", [1, 5, 3000])
def test_star(fg, k):
    g = graphgen.star(k)
    say(f"star k={k}")
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = gpu_raw(fg, off, idx, net=True)
    centre = np.zeros(16, dtype=np.int64)
    centre[[0, 1, 3, 8]] = [1, k, C(k, 2), C(k, 3)]
    leaf = np.zeros(16, dtype=np.int64)
    leaf[[0, 1, 2, 7]] = [1, 1, k - 1, C(k - 1, 2)]
    np.testing.assert_array_equal(f[0], centre)
    np.testing.assert_array_equal(f[1:], np.tile(leaf, (k, 1)))


@pytest.mark.parametrize("n", [4, 5, 1000])
def test_cycle_and_path(fg, n):
    say(f"cycle/path n={n}")
    g = graphgen.cycle(n)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, net=True), oracle.net(off, idx))
    g = graphgen.path(n)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, net=True), oracle.net(off, idx))


# ------------------------------------------------------------------ the small config and medium graphs

def test_er_config(fg):
    """Erdos-Renyi G(2000, 0.005), seed 1: every vertex, raw and net."""
    g = graphgen.erdos_renyi(2000, 0.005, seed=1)
    say("er config")
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    exp = oracle.raw(off, idx)
    np.testing.assert_array_equal(gpu_raw(fg, off, idx), exp)
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, net=True), oracle.raw_to_net(exp))


@pytest.mark.parametrize("plan", list(PLANS))
def test_chung_lu_medium(fg, plan):
    """A 20k-vertex power-law graph (hubs, ragged rows, many tiles)."""
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say(f"chung-lu medium plan={plan} nnz={idx.size}")
    exp = oracle.net(off, idx)
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan], net=True), exp)


def _shuffle_rows(off, idx, seed):
    """The same graph with every row's entries in a seeded random order."""
    rng = np.random.default_rng(seed)
    out = idx.copy()
    for v in range(off.size - 1):
        a, b = int(off[v]), int(off[v + 1])
        if b - a > 1:
            out[a:b] = out[a:b][rng.permutation(b - a)]
    return out


@pytest.mark.parametrize("plan", ["default", "global"])
def test_unsorted_rows(fg, plan):
    """The contract admits rows in any order (fglt_raw relabels and re-sorts
    them): rows shuffled per vertex give the oracle's counts of the sorted
    CSR, a power-law graph with a window tier and a dense graph."""
    for name, g in (("chung-lu 20k", graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)),
                    ("er dense", graphgen.erdos_renyi(300, 0.2, seed=8))):
        off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
        shuffled = _shuffle_rows(off, idx, seed=9)
        assert not np.array_equal(shuffled, idx)
        say(f"unsorted rows: {name} plan={plan}")
        np.testing.assert_array_equal(gpu_raw(fg, off, shuffled, PLANS[plan], net=True), oracle.net(off, idx))


@pytest.mark.parametrize("plan", ["default", "hash", "global"])
@pytest.mark.parametrize("a,b", [(2, 1500), (3, 2600), (40, 300)])
def test_complete_bipartite(fg, plan, a, b):
    """K_{a,b}: the top hub's middles are all b leaves (more than one
    1024-middle chunk for b > 1024), each leaf's wedge ends are the other hubs."""
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    off, idx = csr_arrays(a + b, edges)
    say(f"K_{a},{b} plan={plan}")
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan], net=True), oracle.net(off, idx))


@pytest.mark.parametrize("plan", list(PLANS))
@pytest.mark.parametrize("leaves", [100, 600, 3000])
def test_hub_with_leaves(fg, plan, leaves):
    """A top-ranked hub whose middles are mostly leaves (no wedges below the
    hub) plus a few with wedges: few wedges, many middles."""
    rng = np.random.default_rng(leaves)
    hub, x, y = 0, [1, 2, 3], [4, 5, 6, 7, 8]
    edges = [(hub, xi) for xi in x] + [(xi, yj) for xi in x for yj in y if rng.random() < 0.8]
    edges += [(hub, 9 + k) for k in range(leaves)]
    off, idx = csr_arrays(9 + leaves, edges)
    say(f"hub with {leaves} leaves plan={plan}")
    np.testing.assert_array_equal(gpu_raw(fg, off, idx, PLANS[plan], net=True), oracle.net(off, idx))


@pytest.mark.parametrize("plan", ["default", "hash", "global"])
def test_window_tier_several_windows(fg, plan):
    """150k vertices: ranks span three 65536-rank counter windows, hubs have
    more than 1024 middles (one job per window) and fewer (one job for all
    windows)."""
    g = graphgen.chung_lu(150_000, 2.1, 10.0, 6000.0, seed=11)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say(f"chung-lu 150k plan={plan} nnz={idx.size}")
    st = fg.raw(*to_dev(off, idx), net=True, plan=PLANS[plan], stats=True)
    got, stats = st[0].cpu().numpy(), st[1]
    say(f"c4 tiers {stats['c4_tier_vertices']} wedges {stats['wedge_items_tier']}")
    np.testing.assert_array_equal(got, oracle.net(off, idx))


@pytest.mark.parametrize("rows", [1, 2])
def test_window_tier_row_cuts(fg, rows):
    """The window tier's other ways of cutting a middle's row at the window
    boundaries (the default run above takes the per-entry table): the
    per-vertex table (1) and binary searches of the rows (2)."""
    g = graphgen.chung_lu(150_000, 2.1, 10.0, 6000.0, seed=11)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say(f"chung-lu 150k c4_window_rows={rows}")
    got = gpu_raw(fg, off, idx, {"c4_window_rows": rows}, net=True)
    np.testing.assert_array_equal(got, oracle.net(off, idx))


def test_totals(fg):
    """Graph-level totals: one 20k-vertex graph (several parts per graph,
    device atomics) and a batch of disjoint components, an empty one among
    them (one workgroup per graph)."""
    parts = [graphgen.erdos_renyi(3000, 0.003, seed=51), graphgen.chung_lu(8000, 2.2, 8.0, 300.0, seed=52),
             graphgen.clique(30), graphgen.chung_lu(9000, 2.1, 8.0, 400.0, seed=53)]
    sizes = [p.n for p in parts]
    bounds = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(bounds[-1])
    src = np.concatenate([p.src + bounds[i] for i, p in enumerate(parts)])
    dst = np.concatenate([p.dst + bounds[i] for i, p in enumerate(parts)])
    off, idx = oracle.canonical_csr(n, src, dst)
    f = oracle.net(off, idx)
    say(f"totals: n={n}, components {sizes}")
    net = fg.raw(*to_dev(off, idx), net=True)
    got = fg.totals(net).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.totals(f))
    vo = np.array([0, bounds[1], bounds[1], bounds[2], bounds[3], bounds[4]], dtype=np.int64)  # an empty graph
    got = fg.totals(net, torch.from_numpy(vo).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.totals(f, vo))


def test_stats(fg):
    """Statistics: the triangle total is the sum of the per-vertex triangle
    counts (raw orbit 4) over three; the tiers partition the vertices with work."""
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    raw_e = oracle.raw(off, idx)
    _, st = fg.raw(*to_dev(off, idx), stats=True)
    assert st["triangles"] == int(raw_e[:, 4].sum()) // 3
    assert st["n"] == g.n and st["nnz"] == idx.size
    assert sum(st["wedge_items_tier"]) == st["wedge_items"]
    # vertices with one out-neighbour have merge items but no triangle: no tier takes them
    assert sum(st["tri_items_tier"]) <= st["tri_items"]
    assert st["d_max"] == int(np.diff(off).max())


def test_progress_lines(fg, capfd):
    """FGLT_PROGRESS: each launch segment's end on stderr, in order, the
    finalize last; the counts are those of a call without it."""
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    o, i = to_dev(off, idx)
    want = fg.raw(o, i, net=True).cpu().numpy()
    capfd.readouterr()
    got = fg.raw(o, i, net=True, progress=True)
    torch.cuda.synchronize()
    lines = [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("fglt: ")]
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    names = [m.group(1) for m in (re.match(r"fglt: (\w+) done \(", ln) for ln in lines) if m]
    assert names[0] == "check" and names[-1] == "finalize", lines
    assert names == [s for s in fg._lib.SEGMENTS if s in names], lines  # each once, in launch order


def test_barabasi_albert_and_rmat_small(fg):
    for name, g in [("ba", graphgen.barabasi_albert(5000, 4, seed=8)),
                    ("rmat12", graphgen.rmat(12, 16, 0.57, 0.19, 0.19, seed=9))]:
        off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
        say(f"{name} n={g.n} nnz={idx.size}")
        np.testing.assert_array_equal(gpu_raw(fg, off, idx, net=True), oracle.net(off, idx))


# ------------------------------------------------------------------ properties

def test_net_entry_point(fg):
    g = graphgen.chung_lu(5000, 2.3, 12.0, 500.0, seed=10)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say("fglt_net separate vs fused")
    o, i = to_dev(off, idx)
    r = fg.raw(o, i)
    f_sep = fg.net(r)
    f_fused = fg.raw(o, i, net=True)
    inplace = r.clone()
    fg.net(inplace, out=inplace)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(f_sep.cpu().numpy(), f_fused.cpu().numpy())
    np.testing.assert_array_equal(inplace.cpu().numpy(), f_fused.cpu().numpy())
    exp_raw = oracle.raw(off, idx)
    np.testing.assert_array_equal(fg.net(torch.from_numpy(exp_raw).cuda()).cpu().numpy(), oracle.raw_to_net(exp_raw))


def test_permutation_and_determinism(fg):
    g = graphgen.chung_lu(8000, 2.1, 14.0, 800.0, seed=11)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say("permutation equivariance and reruns")
    f = gpu_raw(fg, off, idx, net=True)
    for _ in range(3):
        np.testing.assert_array_equal(gpu_raw(fg, off, idx, net=True), f)
    perm = np.random.default_rng(1).permutation(g.n)
    off2, idx2 = oracle.canonical_csr(g.n, perm[g.src], perm[g.dst])
    np.testing.assert_array_equal(gpu_raw(fg, off2, idx2, net=True)[perm], f)


# ------------------------------------------------------------------ contract violations

def _status(fg, off, idx):
    o, i = to_dev(off, idx)
    n = off.size - 1
    out = torch.empty((n, 16), dtype=torch.int64, device="cuda")
    try:
        fg.raw(o, i, out=out)
        return 0
    except fg.FgltError as e:
        return e.status


def test_errors(fg):
    say("contract violations")
    off, idx = csr_arrays(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    assert _status(fg, off, idx) == 0
    # asymmetric: drop the entry (1 -> 0)
    o2 = off.copy()
    keep = [k for k in range(idx.size) if not (off[1] <= k < off[2] and idx[k] == 0)]
    bad_idx = idx[keep]
    o2[2:] -= 1
    assert _status(fg, o2, bad_idx) == -2
    # self-loop added symmetrically on vertex 4 (appended to its row)
    sl_idx = np.concatenate([idx, [4]]).astype(np.int32)
    sl_off = off.copy()
    sl_off[5] += 1
    assert _status(fg, sl_off, sl_idx) == -2
    # a repeated entry on both sides: (0,1) twice
    d_idx = np.insert(idx, off[1], 1).astype(np.int32)
    d_off = off.copy()
    d_off[1:] += 1
    d_idx = np.insert(d_idx, d_off[1], 0).astype(np.int32)
    d_off[2:] += 1
    assert _status(fg, d_off, d_idx) == -2
    # an index out of range
    r_idx = idx.copy()
    r_idx[0] = 99
    assert _status(fg, off, r_idx) == -2
    # offsets not monotone
    m_off = off.copy()
    m_off[2] = m_off[3] + 1
    assert _status(fg, m_off, idx) == -2
    # workspace too small, straight through the C ABI (the binding would grow it)
    import ctypes
    o, i = to_dev(off, idx)
    out = torch.empty((5, 16), dtype=torch.int64, device="cuda")
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    L = fg._lib.lib()
    st = L.fglt_raw(5, int(i.numel()), ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(i.data_ptr()),
                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), 64, 0, None, None,
                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -3
    # all isolated
    assert _status(fg, np.zeros(11, np.int64), np.zeros(0, np.int32)) == 0
    f = gpu_raw(fg, np.zeros(11, np.int64), np.zeros(0, np.int32), net=True)
    exp = np.zeros((10, 16), np.int64)
    exp[:, 0] = 1
    np.testing.assert_array_equal(f, exp)


def test_max_degree(fg):
    """The largest admitted degree, 2^21 - 1, at the centre of a star: C(d, 3)
    there is within a factor 6 of the int64 limit and the product
    d (d - 1) (d - 2) just fits; the Sigma_5 transform agrees; one more leaf
    is rejected with FGLT_EOVERFLOW before any counting."""
    k = (1 << 21) - 1
    g = graphgen.star(k)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say(f"star at the degree limit, k={k}")
    f = gpu_raw(fg, off, idx, net=True)
    centre = np.zeros(16, dtype=np.int64)
    centre[[0, 1, 3, 8]] = [1, k, C(k, 2), C(k, 3)]
    leaf = np.zeros(16, dtype=np.int64)
    leaf[[0, 1, 2, 7]] = [1, 1, k - 1, C(k - 1, 2)]
    np.testing.assert_array_equal(f[0], centre)
    assert (f[1:] == leaf).all()
    o, i = to_dev(off, idx)
    f5 = fg.raw(o, i, net=True, sigma5=True)
    torch.cuda.synchronize()
    assert (f5.cpu().numpy() == f[:, :5]).all()
    g = graphgen.star(k + 1)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    say("star one past the degree limit")
    assert _status(fg, off, idx) == -4


# ------------------------------------------------------------------ the transform with Sigma_5

def gpu_sigma5(fg, off, idx, plan=None, net=False):
    o, i = to_dev(off, idx)
    out = fg.raw(o, i, net=net, plan=plan, sigma5=True)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (off.size - 1, 5)
    return out.cpu().numpy()


@pytest.mark.parametrize("plan", ["default", "wave", "block", "global"])
def test_sigma5(fg, plan):
    """FGLT_SIGMA5 ([n][5], Theorem 1) against the oracle's sparse-product
    route, raw and net, with the triangle pass in each tier: the small random
    graphs (a lone vertex, isolated vertices), K_600 and the ER config."""
    graphs = _small_graphs()
    k = graphgen.clique(600)
    graphs.append((k.n, list(zip(k.src.tolist(), k.dst.tolist()))))
    for gi, (n, edges) in enumerate(graphs):
        say(f"sigma5 graph {gi} n={n} m={len(edges)} plan={plan}")
        off, idx = csr_arrays(n, edges)
        np.testing.assert_array_equal(gpu_sigma5(fg, off, idx, PLANS[plan]), oracle.sigma5(off, idx))
        np.testing.assert_array_equal(gpu_sigma5(fg, off, idx, PLANS[plan], net=True), oracle.sigma5(off, idx, net=True))
    g = graphgen.erdos_renyi(2000, 0.005, seed=1)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    np.testing.assert_array_equal(gpu_sigma5(fg, off, idx, PLANS[plan], net=True), oracle.sigma5(off, idx, net=True))


def test_sigma5_medium_and_stats(fg):
    """A 20k-vertex power-law graph against the first five columns of the
    oracle's full transform; statistics and per-segment timing still come back,
    with the skipped segments at zero."""
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    exp = oracle.net(off, idx)[:, :5]
    o, i = to_dev(off, idx)
    out, st = fg.raw(o, i, net=True, sigma5=True, stats=True, timing=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), exp)
    assert st["triangles"] == int(exp[:, 4].sum()) // 3
    seg = st["seg_ms"]
    for name in ("tri2_wave", "tri2_lds", "tri2_global", "l2", "c4_window"):
        assert seg[name] < 0.05, (name, seg[name])


# ------------------------------------------------------------------ sub-dictionaries (Section V)

# index sets that switch each pass on alone and together: degrees and row
# pass 1 only; the triangle pass; row pass 2; the clique pass; the 4-cycle
# pass alone; sets that are and are not closed under Table II
SUBDICTS = [[0, 1, 2, 3, 7, 8], [0, 1, 2, 3, 4, 6, 11], [0, 1, 5, 9, 10, 14], [0, 1, 13, 15], [0, 1, 12],
            [0, 1, 12, 13, 14, 15], [0, 1, 4, 9, 13, 15], [0, 1, 2, 3], [0, 1, 3, 12, 15], [0, 1, 6, 7, 14]]


def gpu_subdict(fg, off, idx, s, plan=None, net=True):
    o, i = to_dev(off, idx)
    out = fg.raw(o, i, net=net, plan=plan, sigma=s)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (off.size - 1, len(s))
    return out.cpu().numpy()


@pytest.mark.parametrize("plan", ["default", "wave", "block", "global"])
def test_subdict(fg, plan):
    """fglt_raw with a sub-dictionary mask against the oracle's U16(s, s)
    conversion of its raw counts, raw-only and net, with every tier plan:
    the small random graphs and K_80."""
    graphs = _small_graphs()
    k = graphgen.clique(80)
    graphs.append((k.n, list(zip(k.src.tolist(), k.dst.tolist()))))
    for gi, (n, edges) in enumerate(graphs):
        off, idx = csr_arrays(n, edges)
        raw = oracle.raw(off, idx)
        for s in SUBDICTS:
            say(f"subdict graph {gi} n={n} m={len(edges)} s={s} plan={plan}")
            np.testing.assert_array_equal(gpu_subdict(fg, off, idx, s, PLANS[plan], net=False),
                                          oracle.subdict(raw, s, net=False))
            np.testing.assert_array_equal(gpu_subdict(fg, off, idx, s, PLANS[plan]), oracle.subdict(raw, s))


def test_subdict_medium_and_skipped_passes(fg):
    """A 20k-vertex power-law graph (window tier included) for every set, and
    timing that shows the skipped passes: no 4-cycle work without orbit 12, no
    clique pass without 13 and 15."""
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    raw = oracle.raw(off, idx)
    o, i = to_dev(off, idx)
    for s in SUBDICTS:
        say(f"subdict medium s={s}")
        out, st = fg.raw(o, i, net=True, sigma=s, stats=True, timing=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.subdict(raw, s))
        seg = st["seg_ms"]
        if 12 not in s:
            assert st["wedge_items"] == 0 and sum(st["c4_tier_vertices"]) == 0
            assert seg["c4_window"] < 0.05
        if 13 not in s and 15 not in s:
            for name in ("tri2_wave", "tri2_lds", "tri2_global"):
                assert seg[name] < 0.05, (s, name, seg[name])
    # the plan's own 4-cycle tiers for orbit 12 alone, window tier included
    out = fg.raw(o, i, net=True, sigma=[0, 1, 12], plan={"c4_wave_max": -1, "c4_block_max": -1, "c4_hash_max": -1})
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.subdict(raw, [0, 1, 12]))


def test_k2b_32bit_window_counters(fg):
    """K_{2,b} with b = 70000: the top hub has b middles and one wedge end
    (the other hub) reached b times, a count beyond 16 bits, so its window job
    takes the 32-bit counters; checked against the closed form (pinned by
    brute force and the oracle on small b)."""
    from tests.test_oracle_pins import k2b_net
    b = 70000
    edges = [(h, 2 + j) for h in (0, 1) for j in range(b)]
    off, idx = csr_arrays(b + 2, edges)
    say(f"K_2,{b}")
    o, i = to_dev(off, idx)
    out, st = fg.raw(o, i, net=True, stats=True)
    torch.cuda.synchronize()
    say(f"c4 tiers {st['c4_tier_vertices']}")
    assert st["c4_tier_vertices"][3] >= 1
    np.testing.assert_array_equal(out.cpu().numpy(), k2b_net(b))


# ------------------------------------------------------------------ asynchronous calls

def test_raw_async_graph_capture(fg):
    """fglt_raw without FGLT_VALIDATE or statistics waits for nothing, so it
    can be captured into a HIP graph on a non-default stream (the second
    stream of the 4-cycle pass forks and joins inside the capture); every
    replay, with eager work and synchronizations between, equals the oracle.
    Chung-Lu 20k (window tier included) and the ER workload."""
    cases = []
    g = graphgen.chung_lu(20_000, 2.1, 16.0, 2000.0, seed=7)
    cases.append(oracle.canonical_csr(g.n, g.src, g.dst))
    g = graphgen.erdos_renyi(2000, 0.005, seed=1)
    cases.append(oracle.canonical_csr(g.n, g.src, g.dst))
    for off, idx in cases:
        n = off.size - 1
        say(f"graph capture of fglt_raw n={n} nnz={idx.size}")
        exp = oracle.net(off, idx)
        o, i = to_dev(off, idx)
        out = torch.empty((n, 16), dtype=torch.int64, device="cuda")
        ws = torch.empty(fg.raw_workspace_bytes(n, idx.size), dtype=torch.uint8, device="cuda")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            fg.raw(o, i, net=True, out=out, workspace=ws, validate=False)  # warm-up: the second stream exists
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            fg.raw(o, i, net=True, out=out, workspace=ws, validate=False)
        for rep in range(3):
            out.fill_(-1)
            graph.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), exp, err_msg=f"replay {rep}")
            assert fg.raw_status(ws) == 0
            _ = torch.ones(1000, device="cuda").sum().item()  # eager work between replays
        del graph


def test_raw_async_status_word(fg):
    """Without FGLT_VALIDATE a malformed CSR returns FGLT_OK at once and the
    device status word tells: an asymmetric graph, an index out of range (no
    kernel reads beyond the arrays), a degree at 2^21; then a good graph on
    the same workspace clears it."""
    L = fg._lib.lib()
    cases = [
        ("asymmetric", np.array([0, 1, 1], np.int64), np.array([1], np.int32), -2),
        ("index out of range", np.array([0, 1, 2], np.int64), np.array([1, 7], np.int32), -2),
        ("offsets beyond the indices", np.array([0, 1, 5], np.int64), np.array([1, 0], np.int32), -2),
    ]
    k = 1 << 21
    g = graphgen.star(k)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    cases.append(("degree 2^21", off, idx, -4))
    ws = torch.empty(fg.raw_workspace_bytes(k + 1, idx.size), dtype=torch.uint8, device="cuda")
    for name, off, idx, want in cases:
        say(f"async status: {name}")
        n = off.size - 1
        o, i = to_dev(off, idx)
        out = torch.empty((n, 16), dtype=torch.int64, device="cuda")
        st = L.fglt_raw(n, idx.size, o.data_ptr(), i.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(), 1,
                        None, None, torch.cuda.current_stream().cuda_stream)
        assert st == 0, name
        assert fg.raw_status(ws) == want, name
        with pytest.raises(fg.FgltError) as e:
            fg.raw(o, i, net=True, workspace=ws)  # validated
        assert e.value.status == want, name
    g = graphgen.erdos_renyi(200, 0.05, seed=2)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    o, i = to_dev(off, idx)
    out = fg.raw(o, i, net=True, workspace=ws, validate=False)
    assert fg.raw_status(ws) == 0
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.net(off, idx))
