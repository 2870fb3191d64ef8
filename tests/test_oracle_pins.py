"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: they use the paper's printed
worked example (Fig. 2), Table II as printed, brute-force enumeration (the
definition), closed forms, walk identities on dense matrix powers, orbit-sum
invariants and networkx's triangle and clique routines.
"""
import math
from itertools import combinations

import networkx as nx
import numpy as np
import pytest

import graphgen
import oracle
from oracle import bruteforce

C = math.comb


def csr_of(n, edges):
    edges = list(edges)
    src = np.array([a for a, b in edges], dtype=np.int64)
    dst = np.array([b for a, b in edges], dtype=np.int64)
    return oracle.canonical_csr(n, src, dst)


def random_graph(rng, n, p):
    return [(i, j) for i, j in combinations(range(n), 2) if rng.random() < p]


# ---------------------------------------------------------------- Fig. 2 / Table II

def test_fig2_oracle(fig2):
    off, idx = csr_of(fig2["n"], fig2["edges"])
    r = oracle.raw(off, idx)
    np.testing.assert_array_equal(r, fig2["raw"])
    np.testing.assert_array_equal(oracle.raw_to_net(r), fig2["net"])


def test_fig2_bruteforce(fig2):
    r, f = bruteforce.frequencies(fig2["n"], fig2["edges"])
    np.testing.assert_array_equal(r, fig2["raw"])
    np.testing.assert_array_equal(f, fig2["net"])


def test_fig2_observations(fig2):
    """The observations printed under Fig. 2: orbit invariance f(v2) = f(v5),
    5 triangles, no induced 4-cycles, claw-free."""
    f = fig2["net"]
    np.testing.assert_array_equal(f[1], f[4])
    assert f[:, 4].sum() // 3 == 5
    assert (f[:, 12] == 0).all()
    assert (f[:, 7] == 0).all() and (f[:, 8] == 0).all()


def test_u16_matches_table2(table2):
    np.testing.assert_array_equal(oracle.U16(), table2)
    # 50 non-zeros (the text's "< 3|Sigma|" bound is not met; the pattern claim is)
    assert np.count_nonzero(table2) == 50


def test_raw_to_net_inverts_table2(table2):
    rng = np.random.default_rng(7)
    f = rng.integers(0, 1000, size=(200, 16)).astype(np.int64)
    rawv = f @ table2.T
    np.testing.assert_array_equal(oracle.raw_to_net(rawv), f)
    # U^{-1} has the same sparsity pattern as U (Section V)
    inv = oracle.raw_to_net(np.eye(16, dtype=np.int64)).T
    np.testing.assert_array_equal(inv @ table2, np.eye(16, dtype=np.int64))
    assert ((inv != 0) == (table2 != 0)).all()


# ---------------------------------------------------------------- brute force

def _edge_cases():
    yield 0, []
    yield 1, []
    yield 2, []
    yield 2, [(0, 1)]
    yield 5, []
    yield 6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)]  # two triangles
    # star K_{1,4} glued to a K4 through the centre
    yield 8, [(0, 1), (0, 2), (0, 3), (0, 4)] + list(combinations([0, 5, 6, 7], 2))
    yield 7, [(0, k) for k in range(1, 7)]  # hub
    yield 6, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)] + [(4, 5)]


@pytest.mark.parametrize("case", list(range(9)))
def test_oracle_vs_bruteforce_edge_cases(case):
    n, edges = list(_edge_cases())[case]
    off, idx = csr_of(n, edges)
    br, bn = bruteforce.frequencies(n, edges)
    r = oracle.raw(off, idx)
    np.testing.assert_array_equal(r, br)
    np.testing.assert_array_equal(oracle.raw_to_net(r), bn)


@pytest.mark.parametrize("seed", list(range(40)))
def test_oracle_vs_bruteforce_random(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 10))
    p = float(rng.choice([0.2, 0.35, 0.5, 0.7, 0.9]))
    edges = random_graph(rng, n, p)
    off, idx = csr_of(n, edges)
    br, bn = bruteforce.frequencies(n, edges)
    r = oracle.raw(off, idx)
    np.testing.assert_array_equal(r, br)
    np.testing.assert_array_equal(oracle.raw_to_net(r), bn)


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", list(range(1, 10)))
def test_clique_closed_form(n):
    g = graphgen.clique(n)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    r = oracle.raw(off, idx)
    f = oracle.raw_to_net(r)
    exp_net = np.zeros(16, dtype=np.int64)
    exp_net[0] = 1
    exp_net[1] = n - 1
    exp_net[4] = C(n - 1, 2)
    exp_net[15] = C(n - 1, 3)
    np.testing.assert_array_equal(f, np.tile(exp_net, (n, 1)))
    a = n - 1
    b = max(n - 2, 0)
    c = max(n - 3, 0)
    exp_raw = [1, a, a * b, C(a, 2), C(a, 2), a * b * c, a * b * c, a * C(b, 2), C(a, 3),
               c * C(a, 2), a * b * c, c * C(a, 2), a * C(b, 2), c * C(a, 2), a * C(b, 2), C(a, 3)]
    np.testing.assert_array_equal(r, np.tile(np.array(exp_raw, dtype=np.int64), (n, 1)))


@pytest.mark.parametrize("k", [1, 2, 3, 5, 9])
def test_star_closed_form(k):
    g = graphgen.star(k)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.net(off, idx)
    centre = np.zeros(16, dtype=np.int64)
    centre[[0, 1, 3, 8]] = [1, k, C(k, 2), C(k, 3)]
    leaf = np.zeros(16, dtype=np.int64)
    leaf[[0, 1, 2, 7]] = [1, 1, k - 1, C(k - 1, 2)]
    np.testing.assert_array_equal(f[0], centre)
    for v in range(1, k + 1):
        np.testing.assert_array_equal(f[v], leaf)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9])
def test_cycle_closed_form(n):
    g = graphgen.cycle(n)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.net(off, idx)
    exp = np.zeros(16, dtype=np.int64)
    exp[0] = 1
    if n == 3:
        exp[[1, 4]] = [2, 1]
    elif n == 4:
        exp[[1, 2, 3, 12]] = [2, 2, 1, 1]
    else:
        exp[[1, 2, 3, 5, 6]] = [2, 2, 1, 2, 2]
    np.testing.assert_array_equal(f, np.tile(exp, (n, 1)))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_path_closed_form(n):
    g = graphgen.path(n)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.net(off, idx)
    for v in range(n):
        a, b = v, n - 1 - v
        exp = np.zeros(16, dtype=np.int64)
        exp[0] = 1
        exp[1] = (a >= 1) + (b >= 1)
        exp[2] = (a >= 2) + (b >= 2)
        exp[3] = (a >= 1) * (b >= 1)
        exp[5] = (a >= 3) + (b >= 3)
        exp[6] = (a >= 1) * (b >= 2) + (a >= 2) * (b >= 1)
        np.testing.assert_array_equal(f[v], exp)


# ---------------------------------------------------------------- walk identities

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_walk_identities(seed):
    rng = np.random.default_rng(seed)
    n = 80
    edges = random_graph(rng, n, 0.12)
    off, idx = csr_of(n, edges)
    r = oracle.raw(off, idx)
    A = np.zeros((n, n), dtype=np.int64)
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    A2 = A @ A
    A3 = A2 @ A
    A4 = A3 @ A
    d = A.sum(1)
    np.testing.assert_array_equal(np.diag(A3), 2 * r[:, 4])
    np.testing.assert_array_equal(np.diag(A4), 2 * r[:, 12] + d * d + r[:, 2])
    # 2-paths from i: walks of length 2 that do not return to i
    np.testing.assert_array_equal(r[:, 2], A2.sum(1) - d)


# ---------------------------------------------------------------- invariants

def _nx_graph(off, idx):
    g = nx.Graph()
    n = off.shape[0] - 1
    g.add_nodes_from(range(n))
    rows = np.repeat(np.arange(n), np.diff(off))
    g.add_edges_from(zip(rows.tolist(), idx.tolist()))
    return g


@pytest.mark.parametrize("which", ["er", "cl", "ba"])
def test_invariants_medium(which):
    if which == "er":
        g = graphgen.erdos_renyi(400, 0.05, seed=11)
    elif which == "cl":
        g = graphgen.chung_lu(1500, 2.1, 12.0, 300.0, seed=12)
    else:
        g = graphgen.barabasi_albert(600, 4, seed=13)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    r = oracle.raw(off, idx)
    f = oracle.raw_to_net(r)
    G = _nx_graph(off, idx)
    tri = nx.triangles(G)
    np.testing.assert_array_equal(r[:, 4], [tri[v] for v in range(g.n)])
    ntri = sum(tri.values()) // 3
    assert f[:, 4].sum() == 3 * ntri
    n_k4 = sum(1 for c in nx.enumerate_all_cliques(G) if len(c) == 4)
    assert f[:, 15].sum() == 4 * n_k4
    S = f.sum(0)
    assert S[2] == 2 * S[3]
    assert S[5] == S[6]
    assert S[7] == 3 * S[8]
    assert 2 * S[9] == S[10] and S[9] == S[11]
    assert S[13] == S[14]
    assert S[12] % 4 == 0 and S[15] % 4 == 0
    assert (f >= 0).all() and (r >= f).all()
    np.testing.assert_array_equal(f @ oracle.U16().T, r)


def test_degrees_and_library_counts():
    g = graphgen.chung_lu(800, 2.3, 10.0, 200.0, seed=21)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    r = oracle.raw(off, idx)
    G = _nx_graph(off, idx)
    np.testing.assert_array_equal(r[:, 1], [G.degree(v) for v in range(g.n)])
    np.testing.assert_array_equal(r[:, 0], 1)


def test_permutation_equivariance():
    g = graphgen.chung_lu(700, 2.2, 10.0, 150.0, seed=31)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.net(off, idx)
    perm = np.random.default_rng(3).permutation(g.n)
    off2, idx2 = oracle.canonical_csr(g.n, perm[g.src], perm[g.dst])
    f2 = oracle.net(off2, idx2)
    np.testing.assert_array_equal(f2[perm], f)


def test_vertex_subset_matches_full():
    g = graphgen.chung_lu(900, 2.1, 12.0, 200.0, seed=41)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    full = oracle.raw(off, idx)
    sel = np.random.default_rng(0).choice(g.n, 50, replace=False)
    np.testing.assert_array_equal(oracle.raw(off, idx, sel), full[sel])


def test_disjoint_union_is_concatenation():
    gs = [graphgen.erdos_renyi(30, 0.3, seed=5, stream=s) for s in range(3)]
    n = sum(g.n for g in gs)
    src, dst, base = [], [], 0
    parts = []
    for g in gs:
        off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
        parts.append(oracle.net(off, idx))
        src.append(g.src.astype(np.int64) + base)
        dst.append(g.dst.astype(np.int64) + base)
        base += g.n
    off, idx = oracle.canonical_csr(n, np.concatenate(src), np.concatenate(dst))
    np.testing.assert_array_equal(oracle.net(off, idx), np.concatenate(parts))


def test_canonical_csr_definition():
    src = np.array([0, 1, 1, 2, 2, 3, 3, 0, 4])
    dst = np.array([1, 0, 1, 3, 3, 2, 0, 3, 4])
    off, idx = oracle.canonical_csr(5, src, dst)
    np.testing.assert_array_equal(off, [0, 2, 3, 4, 6, 6])
    np.testing.assert_array_equal(idx, [1, 3, 0, 3, 0, 2])
    with pytest.raises(ValueError):
        oracle.canonical_csr(3, np.array([0]), np.array([3]))
    off2, idx2 = oracle.canonical_csr_large(5, src, dst)
    np.testing.assert_array_equal(off2, [0, 2, 3, 4, 6, 6])
    np.testing.assert_array_equal(idx2, [1, 3, 0, 3, 0, 2])
    with pytest.raises(ValueError):
        oracle.canonical_csr_large(3, np.array([0]), np.array([3]))


@pytest.mark.parametrize("n,m", [(1, 0), (7, 0), (10, 60), (2000, 30000), (50000, 200000)])
def test_canonical_csr_large_matches_numpy(n, m):
    """The C route for billion-pair graphs against the numpy definition, with
    self-loops and repeated pairs in the input."""
    rng = np.random.default_rng(n + m)
    src = rng.integers(0, n, m)
    dst = np.where(rng.random(m) < 0.05, src, rng.integers(0, n, m))
    a = oracle.canonical_csr(n, src, dst)
    b = oracle.canonical_csr_large(n, src, dst, threads=4)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


# ---------------------------------------------------------------- graph-level totals

@pytest.mark.parametrize("seed", list(range(12)))
def test_totals_vs_bruteforce_copies(seed):
    """Column sums over orbit sizes against a direct count of induced copies."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(3, 10))
    p = float(rng.choice([0.25, 0.5, 0.75]))
    edges = random_graph(rng, n, p)
    off, idx = csr_of(n, edges)
    np.testing.assert_array_equal(oracle.totals(oracle.net(off, idx))[0], bruteforce.graphlet_copies(n, edges))


def test_totals_closed_forms_and_batch():
    C = math.comb
    k6 = graphgen.clique(6)
    st = graphgen.star(5)
    exp_k6 = np.zeros(16, np.int64)
    exp_k6[[0, 1, 4, 15]] = [6, C(6, 2), C(6, 3), C(6, 4)]
    exp_st = np.zeros(16, np.int64)
    exp_st[[0, 1, 2, 3, 7, 8]] = [6, 5, C(5, 2), C(5, 2), C(5, 3), C(5, 3)]
    # the two as one batch: disjoint components, rows 0..5 and 6..11
    n = k6.n + st.n
    src = np.concatenate([k6.src, st.src + k6.n])
    dst = np.concatenate([k6.dst, st.dst + k6.n])
    off, idx = oracle.canonical_csr(n, src, dst)
    t = oracle.totals(oracle.net(off, idx), [0, k6.n, n])
    np.testing.assert_array_equal(t[0], exp_k6)
    np.testing.assert_array_equal(t[1], exp_st)


def test_totals_triangles_match_networkx():
    g = graphgen.chung_lu(800, 2.3, 10.0, 200.0, seed=22)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    t = oracle.totals(oracle.net(off, idx))[0]
    G = _nx_graph(off, idx)
    assert t[4] == sum(nx.triangles(G).values()) // 3
    assert t[1] == G.number_of_edges()


# ---------------------------------------------------------------- the transform with Sigma_5

@pytest.mark.parametrize("seed", list(range(10)))
def test_sigma5_vs_bruteforce(seed):
    """Theorem 1's five orbits against enumeration of every subset of <= 3
    vertices (the brute force's first five columns), raw and net."""
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 10))
    p = float(rng.choice([0.2, 0.5, 0.8, 1.0]))
    edges = random_graph(rng, n, p)
    off, idx = csr_of(n, edges)
    raw, net = bruteforce.frequencies(n, edges)
    np.testing.assert_array_equal(oracle.sigma5(off, idx), raw[:, :5])
    np.testing.assert_array_equal(oracle.sigma5(off, idx, net=True), net[:, :5])


def test_sigma5_closed_forms():
    """K_n: every 2-path closes, so the net path orbits vanish; a star's
    centre holds C(k, 2) bi-forks and its leaves k - 1 paths each; a cycle of
    length >= 4 has no triangle."""
    for n in (1, 2, 3, 7):
        g = graphgen.clique(n)
        off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
        d = n - 1
        np.testing.assert_array_equal(oracle.sigma5(off, idx), np.tile([1, d, d * (d - 1), C(d, 2), C(d, 2)], (n, 1)))
        np.testing.assert_array_equal(oracle.sigma5(off, idx, net=True), np.tile([1, d, 0, 0, C(d, 2)], (n, 1)))
    k = 6
    g = graphgen.star(k)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.sigma5(off, idx, net=True)
    centre = int(np.argmax(np.diff(off)))
    np.testing.assert_array_equal(f[centre], [1, k, 0, C(k, 2), 0])
    leaves = np.delete(f, centre, axis=0)
    np.testing.assert_array_equal(leaves, np.tile([1, 1, k - 1, 0, 0], (k, 1)))
    g = graphgen.cycle(9)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    np.testing.assert_array_equal(oracle.sigma5(off, idx, net=True), np.tile([1, 2, 2, 1, 0], (9, 1)))


@pytest.mark.parametrize("which", ["er", "cl"])
def test_sigma5_matches_full_transform_and_networkx(which):
    """The leading block of Table II is the whole conversion for orbits 0-4:
    the sparse-product route equals the first five columns of the per-vertex
    evaluation of Table I (raw and net), and c3 equals networkx's triangle
    count at each vertex."""
    g = graphgen.erdos_renyi(2000, 0.005, seed=1) if which == "er" else graphgen.chung_lu(3000, 2.2, 12.0, 300.0, seed=5)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    raw = oracle.raw(off, idx)
    np.testing.assert_array_equal(oracle.sigma5(off, idx), raw[:, :5])
    np.testing.assert_array_equal(oracle.sigma5(off, idx, net=True), oracle.raw_to_net(raw)[:, :5])
    tri = nx.triangles(_nx_graph(off, idx))
    np.testing.assert_array_equal(oracle.sigma5(off, idx)[:, 4], [tri[v] for v in range(g.n)])


# ---------------------------------------------------------------- sub-dictionaries (Section V)

def _upward_closed(s, u):
    """Every orbit of s brings every higher orbit its row of U16 reaches."""
    return all(c in s for k in s for c in range(16) if c != k and u[k, c])


# index sets that are closed under Table II (net = those columns of the full net)
CLOSED = [[0, 1], [0, 1, 2, 3, 4], [0, 1, 15], [0, 1, 14, 15], [0, 1, 13, 15], [0, 1, 8, 11, 14, 15],
          [0, 1, 12, 13, 14, 15], [0, 1, 4, 9, 13, 15], list(range(16))]
# and sets that are not (net relative to the sub-dictionary)
OPEN = [[0, 1, 2, 3], [0, 1, 5, 6, 7, 8], [0, 1, 2, 3, 4, 12], [0, 1, 9, 10, 11], [0, 1, 3, 12, 15],
        [0, 1, 5, 13], [0, 1, 6, 7, 14]]


def test_subdict_sets_are_classified(table2):
    for s in CLOSED:
        assert _upward_closed(s, table2), s
    for s in OPEN:
        assert not _upward_closed(s, table2), s
    for bad in ([0, 2, 3], [1, 4], [0], [0, 1, 16]):
        with pytest.raises(ValueError):
            oracle.subdict_columns(bad)


def test_subdict_fig2(fig2):
    """Fig. 2's printed tables: on a closed index set the sub-dictionary's net
    frequencies are the printed net columns; raw-only output is the printed
    raw columns."""
    for s in CLOSED:
        np.testing.assert_array_equal(oracle.subdict(fig2["raw"], s), fig2["net"][:, s])
        np.testing.assert_array_equal(oracle.subdict(fig2["raw"], s, net=False), fig2["raw"][:, s])


def _relative_net(net_bf, s, u):
    """U16(s, s)^{-1} U16(s, :) f for brute-force net frequencies f: what the
    sub-dictionary's conversion gives when the raw counts of s are U16(s, :) f
    (Table II), solved here with exact rational elimination."""
    from fractions import Fraction
    us = [[Fraction(int(u[a, b])) for b in s] for a in s]
    rhs = (u[s, :] @ net_bf.T).T  # [n, |s|] raw counts of s
    out = np.zeros((net_bf.shape[0], len(s)), dtype=np.int64)
    for v in range(net_bf.shape[0]):
        # Gauss-Jordan on the |s| x |s| system
        m = [row[:] + [Fraction(int(rhs[v, a]))] for a, row in enumerate(us)]
        k = len(s)
        for col in range(k):
            piv = next(r for r in range(col, k) if m[r][col] != 0)
            m[col], m[piv] = m[piv], m[col]
            for r in range(k):
                if r != col and m[r][col] != 0:
                    fac = m[r][col] / m[col][col]
                    m[r] = [x - fac * y for x, y in zip(m[r], m[col])]
        for a in range(k):
            x = m[a][k] / m[a][a]
            assert x.denominator == 1
            out[v, a] = int(x)
    return out


@pytest.mark.parametrize("seed", list(range(6)))
def test_subdict_vs_bruteforce(seed, table2):
    """On random small graphs: closed sets give the brute-force net columns;
    every set gives U16(s,s)^{-1} U16(s,:) f for the brute-force net f, and
    raw-only output gives the brute-force raw columns."""
    rng = np.random.default_rng(6000 + seed)
    n = int(rng.integers(5, 10))
    edges = random_graph(rng, n, float(rng.choice([0.4, 0.6, 0.8])))
    off, idx = csr_of(n, edges)
    rbf, fbf = bruteforce.frequencies(n, edges)
    r = oracle.raw(off, idx)
    for s in CLOSED + OPEN:
        np.testing.assert_array_equal(oracle.subdict(r, s, net=False), rbf[:, s])
        got = oracle.subdict(r, s)
        np.testing.assert_array_equal(got, _relative_net(fbf, s, table2))
        if s in CLOSED:
            np.testing.assert_array_equal(got, fbf[:, s])


def test_subdict_open_set_differs_from_full_columns():
    """On K5 a set without the triangle orbit keeps every 2-path: sigma_2 and
    sigma_3 stay raw (12 and 6 per vertex), where the full net has 0."""
    g = graphgen.clique(5)
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    f = oracle.subdict(oracle.raw(off, idx), [0, 1, 2, 3])
    np.testing.assert_array_equal(f, np.tile([1, 4, 12, 6], (5, 1)))


def k2b_net(b):
    """Net frequencies of K_{2,b} (hubs 0, 1; leaves 2 .. b+1): a hub ends b
    2-paths through a leaf to the other hub, centres C(b,2) 2-paths and C(b,3)
    claws over its leaves, and lies on C(b,2) 4-cycles; a leaf centres the
    hub-leaf-hub path, ends 2(b-1) paths, is a claw leaf 2 C(b-1,2) times and
    lies on b-1 4-cycles.  No triangle, paw, diamond or 4-path is induced."""
    hub = np.zeros(16, dtype=np.int64)
    hub[[0, 1, 2, 3, 8, 12]] = [1, b, b, C(b, 2), C(b, 3), C(b, 2)]
    leaf = np.zeros(16, dtype=np.int64)
    leaf[[0, 1, 2, 3, 7, 12]] = [1, 2, 2 * (b - 1), 1, 2 * C(b - 1, 2), b - 1]
    return np.vstack([hub, hub] + [leaf] * b)


@pytest.mark.parametrize("b", [1, 2, 3, 6])
def test_k2b_closed_form(b):
    edges = [(h, 2 + j) for h in (0, 1) for j in range(b)]
    _, net = bruteforce.frequencies(b + 2, edges)
    np.testing.assert_array_equal(net, k2b_net(b))
    off, idx = csr_of(b + 2, edges)
    np.testing.assert_array_equal(oracle.net(off, idx), k2b_net(b))
