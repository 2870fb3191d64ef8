"""Seeded synthetic graph generators (edge lists only).

This module produces raw, uncanonicalised undirected edge lists: pairs
(src, dst) of int32 vertex ids that may contain duplicates, both
directions and self-loops.  It holds none of the graphlet-transform
arithmetic and no CSR construction; every consumer canonicalises the
lists itself (the HIP library with ``fglt_build_csr``, the oracle with
its own plain CPU routine).

Every generator draws from ``numpy.random.Generator(PCG64)`` keyed by a
(seed, stream) pair through ``SeedSequence``, so a (seed, stream) pair
always gives the same graph on the same numpy build.

Workload recipes (the paper measures on LiveJournal and Friendster, which
are not available here; these synthetic families stand in for them):

* Erdos-Renyi G(n, p): every pair i < j independently with probability p.
* Chung-Lu: Pareto weights of shape ``exponent - 1`` capped at ``cap``,
  scale calibrated so that the mean weight equals ``mean_degree``;
  round(sum(w) / 2) endpoint pairs drawn with probability proportional to w.
* R-MAT: ``edge_factor * 2**scale`` pairs, one quadrant draw per bit with
  probabilities (a, b, c, d) and no noise, then a random relabelling (for
  the largest sizes in independently seeded chunks, filled in parallel).
* Barabasi-Albert: grown from a star K_{1,m}; each new vertex links to m
  distinct existing vertices chosen with probability proportional to degree.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for", "EdgeList", "erdos_renyi", "chung_lu", "rmat", "rmat_chunked", "barabasi_albert",
    "batch_graphs", "serving_requests", "star", "clique", "cycle", "path",
]


def rng_for(seed: int, stream: int = 0) -> np.random.Generator:
    """Generator for the (seed, stream) pair."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


@dataclass
class EdgeList:
    """An undirected multigraph given as raw endpoint arrays."""
    n: int
    src: np.ndarray  # int32
    dst: np.ndarray  # int32
    name: str = ""

    @property
    def num_pairs(self) -> int:
        return int(self.src.shape[0])


def _el(n, src, dst, name=""):
    return EdgeList(int(n), np.ascontiguousarray(src, dtype=np.int32),
                    np.ascontiguousarray(dst, dtype=np.int32), name)


def erdos_renyi(n: int, p: float, seed: int, stream: int = 0) -> EdgeList:
    """G(n, p): each of the n(n-1)/2 pairs i < j present with probability p."""
    rng = rng_for(seed, stream)
    if n < 2:
        return _el(n, np.zeros(0), np.zeros(0), f"er({n},{p})")
    # Row-by-row over the strict upper triangle keeps memory at O(n) per step
    # for large n and is exact G(n, p).
    src_parts, dst_parts = [], []
    block = max(1, int(2_000_000 // max(n, 1)))
    for i0 in range(0, n - 1, block):
        i1 = min(n - 1, i0 + block)
        rows = np.arange(i0, i1, dtype=np.int64)
        lens = n - 1 - rows
        tot = int(lens.sum())
        u = rng.random(tot)
        hit = np.nonzero(u < p)[0]
        starts = np.concatenate([[0], np.cumsum(lens)[:-1]])
        r = np.searchsorted(starts, hit, side="right") - 1
        c = rows[r] + 1 + (hit - starts[r])
        src_parts.append(rows[r])
        dst_parts.append(c)
    src = np.concatenate(src_parts) if src_parts else np.zeros(0)
    dst = np.concatenate(dst_parts) if dst_parts else np.zeros(0)
    return _el(n, src, dst, f"er({n},{p})")


def _pareto_weights(rng, n, shape, mean, cap):
    """Capped Pareto weights w = min(x_m * U^(-1/shape), cap) with mean(w) == mean.

    x_m is found by bisection on the realised sample so that the sample mean
    of the capped weights equals ``mean``.
    """
    u = rng.random(n)
    base = np.power(1.0 - u, -1.0 / shape)  # Pareto(1, shape) >= 1

    def mean_for(xm):
        return float(np.minimum(xm * base, cap).mean())

    lo, hi = 1e-6, float(mean)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * base, cap)


def chung_lu(n: int, exponent: float, mean_degree: float, cap: float, seed: int,
             stream: int = 0) -> EdgeList:
    """Edge-sampling Chung-Lu graph with degree exponent ``exponent``.

    Weights follow a Pareto law of shape ``exponent - 1`` (so the degree
    distribution has tail exponent ``exponent``), capped at ``cap`` and scaled
    to mean ``mean_degree``.  round(sum(w)/2) pairs are drawn with both
    endpoints proportional to w; duplicates and self-loops are left in.
    """
    rng = rng_for(seed, stream)
    if n < 2:
        return _el(n, np.zeros(0), np.zeros(0), f"cl({n})")
    w = _pareto_weights(rng, n, exponent - 1.0, mean_degree, cap)
    m_pairs = int(round(w.sum() / 2.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    src = np.empty(m_pairs, dtype=np.int32)
    dst = np.empty(m_pairs, dtype=np.int32)
    chunk = 1 << 22
    for s in range(0, m_pairs, chunk):
        e = min(m_pairs, s + chunk)
        src[s:e] = np.minimum(np.searchsorted(cdf, rng.random(e - s), side="right"), n - 1)
        dst[s:e] = np.minimum(np.searchsorted(cdf, rng.random(e - s), side="right"), n - 1)
    return _el(n, src, dst, f"cl({n},{exponent},{mean_degree},{cap})")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         stream: int = 0, permute: bool = True) -> EdgeList:
    """R-MAT pairs: ``edge_factor * 2**scale`` draws of ``scale`` quadrant bits.

    Quadrant probabilities are (a, b, c, 1-a-b-c) for (top-left, top-right,
    bottom-left, bottom-right); no noise is added.  With ``permute`` the
    vertex ids are relabelled by a uniform random permutation.
    """
    rng = rng_for(seed, stream)
    n = 1 << scale
    m_pairs = edge_factor * n
    t_ab = a + b
    t_abc = a + b + c
    src = np.zeros(m_pairs, dtype=np.int32)
    dst = np.zeros(m_pairs, dtype=np.int32)
    chunk = 1 << 22
    for s in range(0, m_pairs, chunk):
        e = min(m_pairs, s + chunk)
        ss = np.zeros(e - s, dtype=np.int32)
        dd = np.zeros(e - s, dtype=np.int32)
        for bit in range(scale):
            u = rng.random(e - s, dtype=np.float32)
            # quadrant: [0,a) TL, [a,a+b) TR, [a+b,a+b+c) BL, rest BR
            row_bit = (u >= t_ab).astype(np.int32)
            col_bit = (((u >= a) & (u < t_ab)) | (u >= t_abc)).astype(np.int32)
            ss |= row_bit << bit
            dd |= col_bit << bit
        src[s:e] = ss
        dst[s:e] = dd
    if permute:
        perm = rng.permutation(n).astype(np.int32)
        src = perm[src]
        dst = perm[dst]
    return _el(n, src, dst, f"rmat({scale},{edge_factor})")


_RMAT_CHUNK = 1 << 24  # pairs per independently seeded chunk of rmat_chunked


def _rmat_chunk(args):
    """Pairs [k * _RMAT_CHUNK, ...) of rmat_chunked into the shared arrays."""
    from multiprocessing import shared_memory
    k, m_pairs, scale, a, b, c, seed, shm_name, chunk = args
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        both = np.ndarray((2, m_pairs), dtype=np.int32, buffer=shm.buf)
        s = k * chunk
        e = min(m_pairs, s + chunk)
        rng = rng_for(seed, 10_000 + k)
        ss = np.zeros(e - s, dtype=np.int32)
        dd = np.zeros(e - s, dtype=np.int32)
        t_ab, t_abc = a + b, a + b + c
        for bit in range(scale):
            u = rng.random(e - s, dtype=np.float32)
            ss |= (u >= t_ab).astype(np.int32) << bit
            dd |= ((((u >= a) & (u < t_ab)) | (u >= t_abc)).astype(np.int32)) << bit
        both[0, s:e] = ss
        both[1, s:e] = dd
    finally:
        shm.close()
    return k


def rmat_chunked(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
                 workers: int = 16, chunk: int = _RMAT_CHUNK) -> EdgeList:
    """R-MAT pairs as in ``rmat`` (the same quadrant draws, no noise), for
    sizes where one generator stream is too slow: pair chunk k (``chunk``
    pairs, 2^24 by default) draws from stream (seed, 10000 + k), so the result does not depend on
    ``workers`` (processes that fill the chunks side by side); the ids are
    then relabelled by a uniform random permutation from stream (seed, 9999).
    """
    import multiprocessing as mp
    from multiprocessing import shared_memory
    n = 1 << scale
    m_pairs = edge_factor * n
    shm = shared_memory.SharedMemory(create=True, size=2 * 4 * m_pairs)
    try:
        both = np.ndarray((2, m_pairs), dtype=np.int32, buffer=shm.buf)
        jobs = [(k, m_pairs, scale, a, b, c, seed, shm.name, chunk) for k in range((m_pairs + chunk - 1) // chunk)]
        if workers > 1:
            with mp.get_context("fork").Pool(workers) as pool:
                for _ in pool.imap_unordered(_rmat_chunk, jobs):
                    pass
        else:
            for j in jobs:
                _rmat_chunk(j)
        perm = rng_for(seed, 9_999).permutation(n).astype(np.int32)
        src = perm[both[0]]
        dst = perm[both[1]]
        del both
    finally:
        shm.close()
        shm.unlink()
    return _el(n, src, dst, f"rmat_chunked({scale},{edge_factor})")


def barabasi_albert(n: int, m: int, seed: int, stream: int = 0) -> EdgeList:
    """Barabasi-Albert graph grown from the star K_{1,m} (vertices 0..m).

    Each later vertex v links to m distinct earlier vertices drawn with
    probability proportional to their current degree (repeated-endpoint list).
    """
    rng = rng_for(seed, stream)
    m = int(m)
    if n <= m:
        # the seed star itself, truncated
        k = max(0, n - 1)
        return _el(n, np.zeros(k), np.arange(1, k + 1), f"ba({n},{m})")
    total = m + (n - m - 1) * m
    src = np.empty(total, dtype=np.int64)
    dst = np.empty(total, dtype=np.int64)
    ends = np.empty(2 * total, dtype=np.int64)
    src[:m] = 0
    dst[:m] = np.arange(1, m + 1)
    ends[0:2 * m:2] = 0
    ends[1:2 * m:2] = np.arange(1, m + 1)
    ne = 2 * m
    e = m
    u_block = rng.random(8 * m * (n - m) + 64)
    ui = 0
    for v in range(m + 1, n):
        chosen = []
        while len(chosen) < m:
            if ui >= u_block.shape[0]:
                u_block = rng.random(8 * m * (n - m) + 64)
                ui = 0
            t = int(ends[int(u_block[ui] * ne)])
            ui += 1
            if t not in chosen:
                chosen.append(t)
        for t in chosen:
            src[e] = v
            dst[e] = t
            ends[ne] = v
            ends[ne + 1] = t
            ne += 2
            e += 1
    return _el(n, src, dst, f"ba({n},{m})")


def batch_graphs(num_graphs: int, seed: int, n_lo: int = 16, n_hi: int = 512):
    """The mixed small-graph batch: even g Erdos-Renyi, odd g Barabasi-Albert.

    n_g ~ U{n_lo..n_hi}; ER graphs take mean degree k ~ U[2, 12] and
    p = k / (n - 1); BA graphs take m ~ U{1..5}.  Graph g draws from stream g.
    """
    out = []
    for g in range(num_graphs):
        rng = rng_for(seed, 1_000_000 + g)
        n = int(rng.integers(n_lo, n_hi + 1))
        if g % 2 == 0:
            k = float(rng.uniform(2.0, 12.0))
            out.append(erdos_renyi(n, min(1.0, k / max(1, n - 1)), seed, g))
        else:
            mm = int(rng.integers(1, 6))
            out.append(barabasi_albert(n, mm, seed, g))
    return out


def serving_requests(num: int, seed: int, n_lo_exp: float = 3.0, n_hi_exp: float = 6.0,
                     cap: int = 50_000):
    """Request graphs for the serving workload.

    n = round(10^U[n_lo_exp, n_hi_exp]); Chung-Lu with exponent ~ U[2, 3] and
    mean degree ~ U[8, 32]; weight cap min(n - 1, cap).
    """
    out = []
    for r in range(num):
        rng = rng_for(seed, 2_000_000 + r)
        n = int(round(10.0 ** rng.uniform(n_lo_exp, n_hi_exp)))
        expo = float(rng.uniform(2.0, 3.0))
        mean = float(rng.uniform(8.0, 32.0))
        out.append(chung_lu(n, expo, mean, float(min(n - 1, cap)), seed, r))
    return out


def poisson_arrivals(num: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate ``qps``."""
    rng = rng_for(seed, 3_000_000)
    return np.cumsum(rng.exponential(1.0 / qps, size=num))


# Small structured graphs used by closed-form checks.
def star(k: int) -> EdgeList:
    return _el(k + 1, np.zeros(k), np.arange(1, k + 1), f"star({k})")


def clique(n: int) -> EdgeList:
    i, j = np.triu_indices(n, 1)
    return _el(n, i, j, f"K{n}")


def cycle(n: int) -> EdgeList:
    i = np.arange(n)
    return _el(n, i, (i + 1) % n, f"C{n}")


def path(n: int) -> EdgeList:
    i = np.arange(max(0, n - 1))
    return _el(n, i, i + 1, f"P{n}")


# Named workloads (generator parameters only).  Seeds: ER 1, Chung-Lu 2,
# R-MAT 3, batch 4, serving 5.
def make(name: str):
    """The synthetic stand-in for a named workload.

    er       G(n=2000, p=0.005)
    cl       Chung-Lu, n = 1,000,000, degree exponent 2.1, mean degree 20, cap 50,000
    rmat22   R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), ids permuted
    rmat18   the same recipe at scale 18 (a size the oracle finishes in minutes)
    cl_small Chung-Lu, n = 100,000, exponent 2.1, mean 20, cap 5,000
    batch    4096 graphs, n ~ U{16..512}, half ER (mean degree U[2,12]), half BA (m U{1..5})
    rmat26   R-MAT scale 26, edge factor 27, (0.57, 0.19, 0.19, 0.05), ids permuted, chunked
             streams: about 1.8e9 pairs on 67M vertices, the size of the paper's Friendster run
    rmatSc   the chunked recipe at scale S (edge factor 27), e.g. rmat22c .. rmat25c: the
             steps up to the scale-26 run
    """
    if name == "er":
        return erdos_renyi(2000, 0.005, seed=1)
    if name == "cl":
        return chung_lu(1_000_000, 2.1, 20.0, 50_000.0, seed=2)
    if name == "cl_small":
        return chung_lu(100_000, 2.1, 20.0, 5_000.0, seed=2, stream=1)
    if name == "rmat22":
        return rmat(22, 16, 0.57, 0.19, 0.19, seed=3)
    if name == "rmat18":
        return rmat(18, 16, 0.57, 0.19, 0.19, seed=3, stream=1)
    if name == "batch":
        return batch_graphs(4096, seed=4)
    if name == "rmat26":
        return rmat_chunked(26, 27, 0.57, 0.19, 0.19, seed=6)
    if name.startswith("rmat") and name.endswith("c") and name[4:-1].isdigit():
        return rmat_chunked(int(name[4:-1]), 27, 0.57, 0.19, 0.19, seed=6)
    raise KeyError(name)
