"""Writes tests/golden/digests.json: oracle results of the full-size workloads.

For each named workload it generates the graph with ``graphgen``, builds the
canonical CSR and runs the CPU oracle on every vertex, then stores
  - sha256 of the canonical CSR (offsets int64 LE, then indices int32 LE),
  - sha256 of the n x 16 net array (int64 LE, row-major), and its column sums,
  - the oracle's wall time and thread count.
Only ``oracle`` and ``graphgen`` are used; nothing comes from the HIP library.

    python tests/golden/make_digests.py er cl batch rmat18 [--threads N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "digests.json")


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
    return h.hexdigest()


def union_edges(graphs):
    src, dst, base = [], [], 0
    for g in graphs:
        src.append(g.src.astype(np.int64) + base)
        dst.append(g.dst.astype(np.int64) + base)
        base += g.n
    return base, np.concatenate(src), np.concatenate(dst)


def digest(name, threads):
    g = graphgen.make(name)
    if isinstance(g, list):  # batch: the block-diagonal union of the graphs
        n, src, dst = union_edges(g)
    else:
        n, src, dst = g.n, g.src, g.dst
    off, idx = oracle.canonical_csr(n, src, dst)
    t0 = time.time()
    net = oracle.net(off, idx, threads=threads)
    dt = time.time() - t0
    return {
        "n": int(n),
        "nnz": int(idx.size),
        "csr_sha256": sha(off, idx),
        "net_sha256": sha(net),
        "net_colsum": [int(x) for x in net.sum(0)],
        "oracle_seconds": round(dt, 2),
        "oracle_threads": int(threads or oracle.max_threads()),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for name in a.names:
        d = digest(name, a.threads)
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[name] = d
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(name, d, flush=True)


if __name__ == "__main__":
    main()
