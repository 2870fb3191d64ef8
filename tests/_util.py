"""Shared helpers of the test suite (no method arithmetic here)."""
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    """Print and flush, so a GPU step is named before it runs."""
    print(*a, flush=True)
    sys.stdout.flush()


def header_functions():
    """Function names declared in include/fglt.h."""
    text = open(os.path.join(ROOT, "include", "fglt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fglt_[a-z_]+)\s*\(", text)))


def stratified_sample(deg, per_bin, top, seed, max_degree=None):
    """The `top` highest-degree vertices plus up to `per_bin` seeded vertices
    from every log2-degree bin (degree 0 is its own bin)."""
    rng = np.random.default_rng(seed)
    deg = np.asarray(deg)
    order = np.argsort(-deg, kind="stable")
    chosen = [order[:top]] if top else []
    bins = np.where(deg > 0, np.floor(np.log2(np.maximum(deg, 1))).astype(np.int64) + 1, 0)
    for b in np.unique(bins):
        members = np.nonzero(bins == b)[0]
        if max_degree is not None:
            members = members[deg[members] <= max_degree]
        if members.size == 0:
            continue
        k = min(per_bin, members.size)
        chosen.append(rng.choice(members, size=k, replace=False))
    return np.unique(np.concatenate(chosen)) if chosen else np.zeros(0, np.int64)


def csr_arrays(n, edges):
    import oracle
    edges = list(edges)
    src = np.array([a for a, _ in edges], dtype=np.int64)
    dst = np.array([b for _, b in edges], dtype=np.int64)
    return oracle.canonical_csr(n, src, dst)
