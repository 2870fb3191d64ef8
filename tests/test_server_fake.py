"""Scheduling logic of the serving runtime on the CPU (fake executor).

The fake executor computes each request with the CPU oracle and can be made
slow or failing from the host, so admission, skip-ahead, continuous batching,
cancellation, rejection and failure handling are tested without a GPU.
"""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle
from paper_2007_11111_amd.server import Cancelled, Rejected, Server


class FakeStream:
    pass


class FakeExecutor:
    def __init__(self, delay=0.0, fail_rids=(), work_bytes=0):
        self.delay = delay
        self.fail_rids = set(fail_rids)
        self.work_bytes = work_bytes
        self.active = 0
        self.max_active = 0
        self.launches = []
        self._lk = threading.Lock()

    def make_stream(self):
        return FakeStream()

    def bytes_for(self, n, nnz, small):
        return 8 * (n + 1) + 4 * nnz + 128 * n, self.work_bytes

    def _enter(self, reqs):
        with self._lk:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.launches.append([r.rid for r in reqs])
        for r in reqs:
            if r.rid in self.fail_rids:
                with self._lk:
                    self.active -= 1
                raise RuntimeError(f"injected failure on request {r.rid}")
        time.sleep(self.delay)

    def _leave(self):
        with self._lk:
            self.active -= 1

    def run_single(self, req, stream):
        self._enter([req])
        try:
            return [oracle.net(req.offsets, req.indices)]
        finally:
            self._leave()

    def run_batch(self, reqs, stream):
        self._enter(reqs)
        try:
            return [oracle.net(r.offsets, r.indices) for r in reqs]
        finally:
            self._leave()


def _graphs(k, seed, big_every=0):
    out = []
    for i in range(k):
        if big_every and i % big_every == big_every - 1:
            g = graphgen.chung_lu(3000, 2.5, 8.0, 300.0, seed=seed, stream=i)
        else:
            g = graphgen.erdos_renyi(40 + 7 * i, 0.1, seed=seed, stream=i)
        out.append(oracle.canonical_csr(g.n, g.src, g.dst))
    return out


def test_results_match_alone_and_batching_happens():
    ex = FakeExecutor(delay=0.02)
    srv = Server(ex, budget_bytes=1 << 30, streams=2, small_n=512)
    csrs = _graphs(24, seed=1, big_every=6)
    futs = [srv.submit(o, i) for o, i in csrs]
    res = [f.result(timeout=60) for f in futs]
    srv.close()
    for (o, i), r in zip(csrs, res):
        np.testing.assert_array_equal(r.net, oracle.net(o, i))
    assert any(len(l) > 1 for l in ex.launches), "small requests were never batched"
    assert ex.max_active >= 2, "worker streams never overlapped"
    st = srv.stats()
    assert st["completed"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0


def test_budget_blocks_until_release_and_skip_ahead():
    csrs = []
    for n in (40, 400, 30):
        g = graphgen.erdos_renyi(n, 0.1, seed=2, stream=n)
        csrs.append(oracle.canonical_csr(g.n, g.src, g.dst))
    sizes = [8 * (o.size) + 4 * i.size + 128 * (o.size - 1) for o, i in csrs]
    ex = FakeExecutor()
    # room for request 1 alone and for 0 and 2 together, not for 0 and 1
    budget = max(sizes[1], sizes[0] + sizes[2]) + 10
    assert sizes[0] + sizes[1] > budget
    srv = Server(ex, budget_bytes=budget, streams=1, small_n=0)
    f0 = srv.submit(*csrs[0])
    r0 = f0.result(timeout=30)
    f1 = srv.submit(*csrs[1])
    f2 = srv.submit(*csrs[2])
    r2 = f2.result(timeout=30)  # skips ahead of the blocked request 1
    time.sleep(0.2)
    assert not f1.done(), "request 1 ran without budget"
    r0.release()
    r2.release()
    r1 = f1.result(timeout=30)
    r1.release()
    srv.close()
    assert srv.free == budget


def test_oversize_is_rejected():
    ex = FakeExecutor(work_bytes=10 << 20)
    srv = Server(ex, budget_bytes=1 << 20, streams=1)
    o, i = _graphs(1, seed=3)[0]
    with pytest.raises(Rejected):
        srv.submit(o, i).result(timeout=10)
    srv.close()


def test_cancel_queued_request():
    csrs = _graphs(2, seed=4)
    size = [8 * o.size + 4 * i.size + 128 * (o.size - 1) for o, i in csrs]
    ex = FakeExecutor()
    budget = max(size) + 10
    assert sum(size) > budget
    srv = Server(ex, budget_bytes=budget, streams=1, small_n=0)
    r0 = srv.submit(*csrs[0]).result(timeout=30)
    f1 = srv.submit(*csrs[1])  # cannot be admitted while r0 is resident
    assert f1.cancel_request()
    with pytest.raises(Cancelled):
        f1.result(timeout=10)
    r0.release()
    srv.close()


def test_executor_failure_fails_only_its_launch():
    csrs = _graphs(6, seed=5, big_every=1)  # all "big": one request per launch
    ex = FakeExecutor(fail_rids={2})
    srv = Server(ex, budget_bytes=1 << 30, streams=2, small_n=0)
    futs = [srv.submit(o, i) for o, i in csrs]
    for k, f in enumerate(futs):
        if k == 2:
            with pytest.raises(RuntimeError, match="injected"):
                f.result(timeout=30)
        else:
            np.testing.assert_array_equal(f.result(timeout=30).net, oracle.net(*csrs[k]))
    srv.close()
    assert srv.free == (1 << 30) - sum(8 * o.size + 4 * i.size + 128 * (o.size - 1)
                                       for k, (o, i) in enumerate(csrs) if k != 2)


def test_malformed_request_raises_through_future():
    class Raising(FakeExecutor):
        def run_single(self, req, stream):
            raise ValueError("malformed CSR")
    srv = Server(Raising(), budget_bytes=1 << 30, streams=1, small_n=0)
    bad_off = np.array([0, 2, 1], dtype=np.int64)
    bad_idx = np.array([1, 0], dtype=np.int32)
    with pytest.raises(ValueError):
        srv.submit(bad_off, bad_idx).result(timeout=10)
    srv.close()


def test_host_csr_checks_reject_before_the_device():
    from paper_2007_11111_amd import batch_pack, check_host_csr
    good = (np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))
    check_host_csr(*good)
    bad = [
        (np.array([1, 2, 3], np.int64), np.array([1, 0, 0], np.int32)),   # offsets[0] != 0
        (np.array([0, 2, 1, 3], np.int64), np.array([1, 2, 0], np.int32)),  # decreasing
        (np.array([0, 1, 5], np.int64), np.array([1, 0], np.int32)),       # offsets[-1] past the end
        (np.array([0, 1, 1], np.int64), np.array([1, 0], np.int32)),       # offsets[-1] short of the end
        (np.array([-1, 1, 2], np.int64), np.array([1, 0], np.int32)),      # negative start
    ]
    for off, idx in bad:
        with pytest.raises(ValueError):
            check_host_csr(off, idx)
        with pytest.raises(ValueError):
            batch_pack([good, (off, idx)])
    srv = Server(FakeExecutor(), budget_bytes=1 << 30, streams=1)
    for off, idx in bad:
        with pytest.raises(ValueError):
            srv.submit(off, idx).result(timeout=10)
    srv.close()
    assert srv.free == 1 << 30


def test_worker_threads_are_long_lived():
    """One worker thread per stream for the server's lifetime: the number of
    threads does not grow with the number of launches."""
    ex = FakeExecutor()
    before = threading.active_count()
    srv = Server(ex, budget_bytes=1 << 30, streams=3, small_n=0)
    assert srv.num_workers == 3
    csrs = _graphs(30, seed=6)
    for o, i in csrs:
        srv.submit(o, i).result(timeout=30).release()
    assert threading.active_count() <= before + 3
    assert len(ex.launches) == 30
    srv.close()
    assert threading.active_count() <= before


def test_per_request_failure_in_a_batch():
    """An executor outcome that is an exception fails that request alone,
    whether it ran in a batch or by itself."""
    class OneBad(FakeExecutor):
        def run_batch(self, reqs, stream):
            outs = super().run_batch(reqs, stream)
            return [ValueError("bad graph") if r.rid == 1 else o for r, o in zip(reqs, outs)]

        def run_single(self, req, stream):
            outs = super().run_single(req, stream)
            return [ValueError("bad graph")] if req.rid == 1 else outs
    ex = OneBad(delay=0.05)
    srv = Server(ex, budget_bytes=1 << 30, streams=1, small_n=512)
    csrs = _graphs(6, seed=7)
    futs = [srv.submit(o, i) for o, i in csrs]
    for k, f in enumerate(futs):
        if k == 1:
            with pytest.raises(ValueError, match="bad graph"):
                f.result(timeout=30)
        else:
            r = f.result(timeout=30)
            np.testing.assert_array_equal(r.net, oracle.net(*csrs[k]))
            r.release()
    srv.close()
    assert srv.free == 1 << 30
