"""CPU oracle for the fast graphlet transform -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The HIP library and its Python
binding never import, link or call it, and it shares no code with them.

Contents
--------
* ``canonical_csr`` -- the plain definition of a simple undirected graph's
  adjacency (symmetrise, drop self-loops, drop duplicates, sort rows), in numpy;
  ``canonical_csr_large`` the same in C with OpenMP, for billions of pairs.
* ``raw`` / ``net`` / ``raw_to_net`` -- ctypes front end of ``fglt_oracle.c``,
  the per-vertex evaluation of Table I and the back-substitution with Table II.
* ``bruteforce`` (module) -- enumeration of every vertex subset of size <= 4,
  the definition of raw and net frequencies, for tiny graphs.
* ``U16`` -- Table II as a dense integer matrix.
* ``sigma5`` -- the transform with the sub-dictionary Sigma_5 (Theorem 1) by
  sparse matrix products, independent of ``raw``.
* ``totals`` -- graph-level induced-graphlet counts from net frequencies.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fglt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

NORB = 16


def build(force: bool = False) -> str:
    """Compile fglt_oracle.c with gcc -O2 -fopenmp into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            lib = ctypes.CDLL(path)
            p64 = ctypes.POINTER(ctypes.c_int64)
            p32 = ctypes.POINTER(ctypes.c_int32)
            lib.oracle_raw.argtypes = [ctypes.c_int64, p64, p32, ctypes.c_int64, p64, p64, ctypes.c_int]
            lib.oracle_raw.restype = ctypes.c_int
            lib.oracle_raw_to_net.argtypes = [ctypes.c_int64, p64, p64]
            lib.oracle_raw_to_net.restype = None
            lib.oracle_u16.argtypes = [p64]
            lib.oracle_u16.restype = None
            lib.oracle_canonical_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, p32, p32, p64, p32, ctypes.c_int]
            lib.oracle_canonical_csr.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def canonical_csr(n: int, src, dst):
    """Adjacency of the simple undirected graph on n vertices spanned by the
    pairs (src[t], dst[t]): both directions, self-loops and duplicates
    removed, rows sorted.  Returns (offsets int64[n+1], indices int32[nnz])."""
    n = int(n)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("vertex id out of range")
    s = np.concatenate([src, dst])
    d = np.concatenate([dst, src])
    keep = s != d
    key = np.unique(s[keep] * max(n, 1) + d[keep])
    rows = key // max(n, 1)
    cols = key % max(n, 1)
    offsets = np.zeros(n + 1, dtype=np.int64)
    if n:
        np.cumsum(np.bincount(rows, minlength=n), out=offsets[1:])
    return offsets, cols.astype(np.int32)


def canonical_csr_large(n: int, src, dst, threads: int = 0):
    """``canonical_csr`` for graphs of billions of pairs: the same definition
    by the C routine (rows filled in parallel, then sorted and deduplicated
    row by row), with int32 ids.  Returns (offsets int64[n+1], indices
    int32[nnz]); the indices are a view of a 2m-entry buffer."""
    n = int(n)
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    off = np.zeros(n + 1, dtype=np.int64)
    idx = np.empty(max(2 * s.size, 1), dtype=np.int32)
    st = _load().oracle_canonical_csr(n, s.size, _p32(s) if s.size else _p32(np.zeros(1, np.int32)),
                                      _p32(d) if d.size else _p32(np.zeros(1, np.int32)), _p64(off), _p32(idx),
                                      int(threads))
    if st == -3:
        raise ValueError("vertex id out of range")
    if st != 0:
        raise RuntimeError(f"oracle_canonical_csr failed with status {st}")
    return off, idx[:off[-1]]


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def raw(offsets, indices, vertices=None, threads: int = 0) -> np.ndarray:
    """Raw frequencies (Table I) of the selected vertices (all if None)."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    n = off.shape[0] - 1
    if vertices is None:
        nsel = n
        sel_ptr = ctypes.POINTER(ctypes.c_int64)()
    else:
        sel = np.ascontiguousarray(vertices, dtype=np.int64)
        if sel.size and (sel.min() < 0 or sel.max() >= n):
            raise ValueError("vertex out of range")
        nsel = sel.shape[0]
        sel_ptr = _p64(sel)
    out = np.zeros((max(nsel, 0), NORB), dtype=np.int64)
    if idx.size == 0:
        idx = np.zeros(1, dtype=np.int32)
    st = lib.oracle_raw(n, _p64(off), _p32(idx), nsel, sel_ptr, _p64(out), int(threads))
    if st != 0:
        raise RuntimeError(f"oracle_raw failed with status {st}")
    return out


def raw_to_net(raw_counts) -> np.ndarray:
    """Back-substitution with U16 (Table II), row by row."""
    lib = _load()
    r = np.ascontiguousarray(raw_counts, dtype=np.int64).reshape(-1, NORB)
    out = np.zeros_like(r)
    lib.oracle_raw_to_net(r.shape[0], _p64(r), _p64(out))
    return out


def net(offsets, indices, vertices=None, threads: int = 0) -> np.ndarray:
    """Net frequencies: Table I followed by Table II."""
    return raw_to_net(raw(offsets, indices, vertices, threads))


def sigma5(offsets, indices, net: bool = False) -> np.ndarray:
    """The transform with the sub-dictionary Sigma_5 (the section on the
    transform with Sigma_5, Theorem 1), by its own route and not through
    ``raw``: with the adjacency matrix A (scipy's sparse product as the one
    library step) d0 = e, d1 = p1 = A e, d2 = p2 = A p1 - p1,
    d3 = p1 (p1 - 1) / 2 and d4 = c3 = (A .* A^2) e / 2, the triangles at each
    vertex; net by the leading 5x5 block of Table II (f2 = d2 - 2 c3,
    f3 = d3 - c3).  [n, 5] int64.  A^2 is formed whole, so this is for small
    and medium graphs."""
    import scipy.sparse as sp

    off = np.asarray(offsets, dtype=np.int64)
    idx = np.asarray(indices, dtype=np.int64)
    n = off.size - 1
    A = sp.csr_matrix((np.ones(idx.size, dtype=np.int64), idx, off), shape=(n, n))
    e = np.ones(n, dtype=np.int64)
    p1 = A @ e
    p2 = A @ p1 - p1
    c3 = np.asarray(A.multiply(A @ A).sum(axis=1), dtype=np.int64).reshape(n)
    assert np.all(c3 % 2 == 0)
    c3 //= 2
    out = np.stack([e, p1, p2, p1 * (p1 - 1) // 2, c3], axis=1).astype(np.int64)
    if net:
        out[:, 2] -= 2 * c3
        out[:, 3] -= c3
    return out


# Fig. 1: how many vertices of orbit k's graphlet lie in orbit k (node;
# edge; P3 ends, centre; triangle; P4 ends, inner; claw leaves, centre; paw
# tip, base, centre; 4-cycle; diamond off-cord, on-cord; 4-clique).
ORBIT_NODES = np.array([1, 2, 2, 1, 3, 2, 2, 3, 1, 1, 2, 1, 4, 2, 2, 4], dtype=np.int64)


def totals(net_counts, vtx_offsets=None) -> np.ndarray:
    """Graph-level totals: for each graph g (rows vtx_offsets[g] ..
    vtx_offsets[g+1]-1 of the net frequencies; one graph when None) and orbit
    k, the sum of the net frequencies of orbit k over the graph divided by
    the orbit's vertex count in its graphlet -- the number of induced copies
    of that graphlet (each copy is counted at every vertex it holds in orbit
    k).  [G, 16] int64."""
    f = np.ascontiguousarray(net_counts, dtype=np.int64).reshape(-1, NORB)
    if vtx_offsets is None:
        vtx_offsets = [0, f.shape[0]]
    off = np.asarray(vtx_offsets, dtype=np.int64)
    out = np.zeros((off.size - 1, NORB), dtype=np.int64)
    for g in range(off.size - 1):
        col = f[off[g]:off[g + 1]].sum(axis=0)
        assert np.all(col % ORBIT_NODES == 0), "net frequencies whose orbit sums do not divide"
        out[g] = col // ORBIT_NODES
    return out


def U16() -> np.ndarray:
    """Table II, U16 f = raw, as a dense 16x16 int64 matrix."""
    u = np.zeros((NORB, NORB), dtype=np.int64)
    _load().oracle_u16(_p64(u))
    return u


def subdict_columns(mask) -> list:
    """The index set s of a sub-dictionary, ascending, from a 16-bit mask or
    an iterable of orbit numbers.  Table II's caption admits any s with
    {0, 1} <= s <= {0, ..., 15}."""
    if isinstance(mask, (int, np.integer)):
        s = [k for k in range(NORB) if (int(mask) >> k) & 1]
    else:
        s = sorted({int(k) for k in mask})
    if not s or s[0] != 0 or (len(s) < 2 or s[1] != 1) or s[-1] >= NORB:
        raise ValueError(f"a sub-dictionary must contain orbits 0 and 1 and lie in 0..15: {s}")
    return s


def subdict(raw_counts, mask, net: bool = True) -> np.ndarray:
    """The transform with the sub-dictionary of index set s (Section V: the
    conversion of a sub-dictionary is the sub-matrix U16(s, s) of Table II).
    From the 16 raw frequencies of each vertex it keeps the columns s; with
    ``net`` it solves U16(s, s) f_s = raw_s by back-substitution from the
    highest orbit down (U16(s, s) is unit upper triangular, so the solve is
    exact in integers).  [rows, |s|] int64, columns in ascending orbit order."""
    s = subdict_columns(mask)
    r = np.ascontiguousarray(raw_counts, dtype=np.int64).reshape(-1, NORB)
    out = r[:, s].copy()
    if not net:
        return out
    u = U16()[np.ix_(s, s)]
    for a in range(len(s) - 1, -1, -1):
        for b in range(a + 1, len(s)):
            if u[a, b]:
                out[:, a] -= u[a, b] * out[:, b]
    return out
