"""Brute-force graphlet frequencies by enumeration -- TEST INFRASTRUCTURE ONLY.

The definitions (Sections II and IV of the paper): for a vertex v and a
graphlet sigma_k of the dictionary Sigma_16 (all connected graphs on at most
four vertices, each with a designated incidence orbit),

* the raw frequency  \\hat d_k(v) counts the sigma_k-pattern subgraphs
  (a vertex set S containing v together with a subset F of the edges of
  G[S], with (S, F) connected, spanning and isomorphic to sigma_k) in which
  v sits at the designated orbit -- induced or not;
* the net frequency d_k(v) counts only the induced ones (F = all edges of
  G[S]); for a complete, non-redundant family these are the induced-subgraph
  counts, which is what the conversion of Table II recovers.

The graphlet of (S, F) and v's orbit in it follow from Table I's names and
the ordering rules of the Fig. 1 caption (vertices, then edges, then the
degree of the incidence node, the 4-cycle excepted):

  |S| = 1: sigma_0.  |S| = 2: sigma_1.
  |S| = 3: two edges -> sigma_2 (v an end, degree 1) / sigma_3 (v the root);
           three edges -> sigma_4.
  |S| = 4, three edges: claw -> sigma_7 (leaf) / sigma_8 (centre);
                        3-path -> sigma_5 (end) / sigma_6 (interior).
  |S| = 4, four edges: 4-cycle -> sigma_12; paw -> sigma_9 (handle tip,
           degree 1) / sigma_10 (base, degree 2) / sigma_11 (centre, degree 3).
  |S| = 4, five edges (diamond): sigma_13 (off-cord, degree 2) /
           sigma_14 (on-cord, degree 3).
  |S| = 4, six edges: sigma_15.

Cost is exponential in the subset size and the edge-subset count; use only
for graphs of a few dozen vertices at most.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

NORB = 16


def graphlet_copies(n: int, edges) -> np.ndarray:
    """For each orbit k, the number of induced copies of orbit k's graphlet:
    connected vertex sets S (|S| <= 4) whose induced subgraph puts some vertex
    at orbit k, by enumeration (no orbit sizes are involved)."""
    es = _edge_set(n, edges)
    out = np.zeros(NORB, dtype=np.int64)
    out[0] = n
    for size in (2, 3, 4):
        for S in combinations(range(n), size):
            induced = [(a, b) for a, b in combinations(S, 2) if (a, b) in es]
            if not _connected(S, induced):
                continue
            for k in {orbit_of(v, S, induced) for v in S}:
                out[k] += 1
    return out


def orbit_of(v, verts, edges) -> int:
    """Index k of the graphlet/orbit of vertex v in the connected spanning
    graph (verts, edges); edges is a list of 2-tuples."""
    k = len(verts)
    deg = {x: 0 for x in verts}
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
    ne = len(edges)
    dv = deg[v]
    if k == 1:
        return 0
    if k == 2:
        return 1
    if k == 3:
        if ne == 3:
            return 4
        return 2 if dv == 1 else 3
    # k == 4
    if ne == 3:
        if max(deg.values()) == 3:  # claw
            return 7 if dv == 1 else 8
        return 5 if dv == 1 else 6  # 3-path
    if ne == 4:
        if all(d == 2 for d in deg.values()):
            return 12
        return {1: 9, 2: 10, 3: 11}[dv]  # paw
    if ne == 5:
        return 13 if dv == 2 else 14
    return 15


def _connected(verts, edges) -> bool:
    verts = list(verts)
    if len(verts) <= 1:
        return True
    adj = {x: [] for x in verts}
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {verts[0]}
    stack = [verts[0]]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == len(verts)


def _edge_set(n, edges):
    es = set()
    for a, b in edges:
        a, b = int(a), int(b)
        if a == b:
            continue
        es.add((min(a, b), max(a, b)))
    return es


def frequencies(n: int, edges):
    """(raw, net) int64 arrays of shape (n, 16) by full enumeration.

    ``edges`` is any iterable of vertex pairs; duplicates, both directions and
    self-loops are ignored, so the graph is the simple undirected one."""
    es = _edge_set(n, edges)
    raw = np.zeros((n, NORB), dtype=np.int64)
    net = np.zeros((n, NORB), dtype=np.int64)
    for v in range(n):
        raw[v, 0] = net[v, 0] = 1
    for size in (2, 3, 4):
        for S in combinations(range(n), size):
            induced = [(a, b) for a, b in combinations(S, 2) if (a, b) in es]
            if not _connected(S, induced):
                continue
            # net: the induced subgraph
            for v in S:
                net[v, orbit_of(v, S, induced)] += 1
            # raw: every spanning connected edge subset
            ne = len(induced)
            for mask in range(1, 1 << ne):
                F = [induced[t] for t in range(ne) if mask >> t & 1]
                if len(F) < size - 1 or not _connected(S, F):
                    continue
                for v in S:
                    raw[v, orbit_of(v, S, F)] += 1
    return raw, net
