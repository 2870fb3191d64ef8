"""The serving front end on the GPU: requests of mixed sizes through Server
and GpuExecutor (fglt_batch for n <= 512, fglt_raw otherwise), each result
equal to the oracle's net frequencies of that request alone."""
import numpy as np
import pytest

import graphgen
import oracle
from tests._util import say

pytestmark = pytest.mark.gpu


def _serve(csrs, copy_out=False, budget=8 << 30, streams=4):
    from paper_2007_11111_amd.server import GpuExecutor, Server
    srv = Server(GpuExecutor(copy_out=copy_out), budget_bytes=budget, streams=streams)
    try:
        futs = [srv.submit(o, i) for o, i in csrs]
        res = [f.result(timeout=120) for f in futs]
    finally:
        srv.close()
    return srv, res


def test_server_mixed_requests():
    gs = graphgen.serving_requests(24, seed=5, n_lo_exp=1.3, n_hi_exp=3.6)
    csrs = [oracle.canonical_csr(g.n, g.src, g.dst) for g in gs]
    sizes = [o.size - 1 for o, _ in csrs]
    assert min(sizes) <= 512 < max(sizes)
    say(f"server: {len(csrs)} requests, n from {min(sizes)} to {max(sizes)}")
    srv, res = _serve(csrs)
    for k, ((o, i), r) in enumerate(zip(csrs, res)):
        got = r.net.cpu().numpy()
        # the request's CSR stays resident on the device with its result
        lo, li = r.local_csr()
        np.testing.assert_array_equal(lo.cpu().numpy(), o)
        np.testing.assert_array_equal(li.cpu().numpy(), i)
        r.release()
        np.testing.assert_array_equal(got, oracle.net(o, i), err_msg=f"request {k} (n={o.size - 1})")
    assert srv.free == 8 << 30
    st = srv.stats()
    assert st["completed"] == len(csrs) and st["p99_ms"] >= st["p50_ms"] > 0


def test_server_requests_up_to_1e5_vertices():
    """Requests of the serving recipe with n up to 10^5 (and a few small ones),
    in the mix and with the results copied to the host, each equal to the
    oracle alone."""
    gs = graphgen.serving_requests(10, seed=15, n_lo_exp=3.0, n_hi_exp=5.0)
    gs += graphgen.serving_requests(6, seed=16, n_lo_exp=1.5, n_hi_exp=2.6)
    csrs = [oracle.canonical_csr(g.n, g.src, g.dst) for g in gs]
    sizes = [o.size - 1 for o, _ in csrs]
    say(f"server large: {len(csrs)} requests, n from {min(sizes)} to {max(sizes)}")
    assert max(sizes) >= 30000
    srv, res = _serve(csrs, copy_out=True, budget=32 << 30)
    for k, ((o, i), r) in enumerate(zip(csrs, res)):
        assert r.host_net is not None and r.latency_host_s >= r.latency_s > 0
        np.testing.assert_array_equal(r.host_net, oracle.net(o, i), err_msg=f"request {k} (n={o.size - 1})")
        r.release()
    assert srv.free == 32 << 30
