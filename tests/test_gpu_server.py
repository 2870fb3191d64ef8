"""The serving front end on the GPU: requests of mixed sizes through Server
and GpuExecutor (fglt_batch for n <= 512, fglt_raw otherwise), each result
equal to the oracle's net frequencies of that request alone."""
import numpy as np
import pytest

import graphgen
import oracle
from tests._util import say

pytestmark = pytest.mark.gpu


def test_server_mixed_requests():
    from paper_2007_11111_amd.server import GpuExecutor, Server
    gs = graphgen.serving_requests(24, seed=5, n_lo_exp=1.3, n_hi_exp=3.6)
    csrs = [oracle.canonical_csr(g.n, g.src, g.dst) for g in gs]
    sizes = [o.size - 1 for o, _ in csrs]
    assert min(sizes) <= 512 < max(sizes)
    say(f"server: {len(csrs)} requests, n from {min(sizes)} to {max(sizes)}")
    srv = Server(GpuExecutor(), budget_bytes=8 << 30, streams=4)
    try:
        futs = [srv.submit(o, i) for o, i in csrs]
        res = [f.result(timeout=60) for f in futs]
    finally:
        srv.close()
    for k, ((o, i), r) in enumerate(zip(csrs, res)):
        got = r.net.cpu().numpy()
        r.release()
        np.testing.assert_array_equal(got, oracle.net(o, i), err_msg=f"request {k} (n={o.size - 1})")
    assert srv.free == 8 << 30
    st = srv.stats()
    assert st["completed"] == len(csrs) and st["p99_ms"] >= st["p50_ms"] > 0
