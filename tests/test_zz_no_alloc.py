"""fglt_raw_noalloc (the transform on the library's own device array) through
the C ABI against fglt_raw with a caller workspace: two calls in a row, the
second on a smaller graph, then a sub-dictionary, raw-only output and the
size limit."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2007_11111_amd as fg
    assert torch.cuda.is_available()
    L = fg._lib.lib()
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.fglt_raw_noalloc.argtypes = [i64, i64, vp, vp, vp, ctypes.c_uint, vp, vp, vp]
    L.fglt_raw_noalloc.restype = ctypes.c_int
    return fg, L


def _noalloc(fg, L, off, idx, flags, cols):
    n, nnz = off.numel() - 1, idx.numel()
    out = torch.full((n, cols), -7, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    st = L.fglt_raw_noalloc(n, nnz, off.data_ptr(), idx.data_ptr() if nnz else None, out.data_ptr(), flags,
                            None, None, s)
    torch.cuda.synchronize()
    return st, out


def _dev(g):
    off, idx = oracle.canonical_csr(g.n, g.src, g.dst)
    return torch.from_numpy(off).cuda(), torch.from_numpy(idx).cuda()


def test_noalloc_matches_fglt_raw(lib):
    fg, L = lib
    from paper_2007_11111_amd._lib import FGLT_NET, FGLT_SIGMA
    big = graphgen.chung_lu(60_000, 2.1, 16.0, 3000.0, seed=11)   # window tier included
    small = graphgen.erdos_renyi(2000, 0.005, seed=1)
    for name, g in (("chung-lu 60k", big), ("erdos-renyi 2000", small)):
        off, idx = _dev(g)
        say(f"noalloc {name}: n={g.n} nnz={idx.numel()}")
        st, got = _noalloc(fg, L, off, idx, FGLT_NET, 16)
        assert st == 0, fg._lib.STATUS.get(st, st)
        exp = fg.raw(off, idx, net=True)
        torch.cuda.synchronize()
        assert torch.equal(got, exp)
    # raw-only and a sub-dictionary on the smaller graph, after the larger one
    st, got = _noalloc(fg, L, off, idx, 0, 16)
    assert st == 0 and torch.equal(got, fg.raw(off, idx))
    st, got = _noalloc(fg, L, off, idx, FGLT_NET | FGLT_SIGMA(0x5FFF), 14)
    assert st == 0 and torch.equal(got, fg.raw(off, idx, net=True, sigma=0x5FFF))


def test_noalloc_limits(lib):
    fg, L = lib
    from paper_2007_11111_amd._lib import FGLT_TIMING
    g = graphgen.erdos_renyi(2000, 0.005, seed=1)
    off, idx = _dev(g)
    st, _ = _noalloc(fg, L, off, idx, FGLT_TIMING, 16)
    assert st == -1
    # a graph whose workspace exceeds the array: rejected before any launch
    n, nnz = 4_000_000, 40_000_000
    assert int(L.fglt_raw_workspace(n, nnz)) > 256 << 20
    st = L.fglt_raw_noalloc(n, nnz, off.data_ptr(), idx.data_ptr(), off.data_ptr(), 0, None, None, None)
    assert st == -3
    # the empty graph
    e = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert L.fglt_raw_noalloc(0, 0, e.data_ptr(), None, e.data_ptr(), 1, None, None, None) == 0
