"""Serving runtime: continuous batching of graphlet-transform requests.

A request is one graph (host CSR).  The server
  * admits requests by an HBM budget: the bytes a request holds on the device
    (its CSR, its n x 16 result, and -- while it runs -- its workspace) must
    fit the free budget; a request larger than the whole budget is rejected;
  * keeps admitted CSRs and results resident on the device until the client
    releases them (the budget is returned then);
  * batches continuously: one long-lived worker thread per HIP stream; when a
    worker is free it takes the waiting requests in arrival order (skipping
    ahead past a request that does not fit yet) and either packs the small
    graphs (n <= small_n) into one fglt_batch launch or hands one large graph
    to fglt_raw; the workers' streams run at once, so their work overlaps on
    the GPU;
  * records per-request latency from arrival to the completion of its
    kernels (and, with a copying executor, to the end of the copy of its
    result to the host).

The device work goes through an executor object; ``GpuExecutor`` calls the HIP
library.  Tests substitute a CPU executor to drive the scheduling logic
without a GPU.  An executor returns one outcome per request of a launch: the
result, or an exception that fails that request alone; an exception raised
by the executor fails the whole launch.
"""
from __future__ import annotations

import itertools
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

NORB = 16


class Rejected(Exception):
    """The request can never be admitted (larger than the whole budget)."""


class Cancelled(Exception):
    """The request was cancelled before it started."""


@dataclass
class Request:
    rid: int
    offsets: np.ndarray      # host int64 [n+1]
    indices: np.ndarray      # host int32 [nnz]
    arrival: float           # time.perf_counter() at submission
    future: Future = field(default_factory=Future)
    bytes_resident: int = 0  # CSR + result
    bytes_work: int = 0      # workspace while running
    start: float = 0.0
    end: float = 0.0

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])


@dataclass
class Outcome:
    """What an executor returns for one request."""
    net: object                # device tensor (GpuExecutor) or ndarray; n x 16 int64
    csr: object = None         # the request's resident device CSR (offsets, indices), if kept
    host_net: object = None    # the result copied to the host (copying executors)
    t_done: float = 0.0        # perf_counter() when its kernels had completed
    t_host: float = 0.0        # perf_counter() when its host copy had completed
    csr_base: tuple = (0, 0)   # (vertex, entry) offset of that CSR inside a batch's packed CSR


@dataclass
class Result:
    rid: int
    net: object              # device tensor (GpuExecutor) or ndarray; n x 16 int64
    latency_s: float         # arrival -> kernels complete
    queued_s: float          # arrival -> start of its launch
    batched_with: int        # number of requests in the same launch
    latency_host_s: float = 0.0  # arrival -> result on the host (copying executors), else 0
    csr: object = None       # resident device CSR (views into the launch's packed CSR for a batch)
    host_net: object = None
    _server: "Server" = None
    csr_base: tuple = (0, 0)

    def local_csr(self):
        """The request's resident CSR in its own vertex numbering (a batched
        request's views hold the packed batch's global ids and offsets)."""
        off, idx = self.csr
        v0, e0 = self.csr_base
        return (off - e0, idx - v0) if (v0 or e0) else (off, idx)

    def release(self):
        """Returns the request's resident bytes to the budget."""
        if self._server is not None:
            self._server._release(self.rid)
            self._server = None
            self.net = None
            self.csr = None


class GpuExecutor:
    """Runs requests on the GPU through the C ABI (one HIP stream per worker).

    The request's CSR is copied to the device and kept there with its result
    until release; with copy_out=True the result is also copied to host
    memory and the time of that copy is recorded."""

    def __init__(self, device=0, batch_plan=None, copy_out=False):
        import torch
        import paper_2007_11111_amd as fg
        self.torch = torch
        self.fg = fg
        self.device = torch.device("cuda", device)
        self.batch_plan = batch_plan
        self.copy_out = copy_out

    def make_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def bytes_for(self, n, nnz, small):
        csr = 8 * (n + 1) + 4 * nnz
        out = 8 * NORB * n
        if small:
            work = int(self.fg._lib.lib().fglt_batch_workspace(1, n, nnz))
        else:
            work = self.fg.raw_workspace_bytes(n, nnz)
        return csr + out, work

    def _finish(self, stream, nets, csrs, bases=None):
        stream.synchronize()
        t_done = time.perf_counter()
        hosts = [None] * len(nets)
        t_host = 0.0
        if self.copy_out:
            # into pageable memory: pinned buffers would stay pinned for as long
            # as the client keeps the result
            with self.torch.cuda.stream(stream):
                hosts = [x.to("cpu") if not isinstance(x, Exception) else None for x in nets]
            t_host = time.perf_counter()
            hosts = [h.numpy() if h is not None else None for h in hosts]
        bases = bases or [(0, 0)] * len(nets)
        return [x if isinstance(x, Exception) else Outcome(x, c, h, t_done, t_host, bb)
                for x, c, h, bb in zip(nets, csrs, hosts, bases)]

    def run_single(self, req, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            off = torch.from_numpy(req.offsets).to(self.device, non_blocking=True)
            idx = torch.from_numpy(req.indices).to(self.device, non_blocking=True)
            n, nnz = int(off.numel()) - 1, int(idx.numel())
            ws = torch.empty(max(self.fg.raw_workspace_bytes(n, nnz), 1), dtype=torch.uint8, device=self.device)
            try:
                # enqueued without waiting; the status word is read once the stream is done
                out = self.fg.transform(off, idx, workspace=ws, validate=False, stream=stream)
            except self.fg.FgltError as e:
                stream.synchronize()
                return [e]
        st = self.fg.raw_status(ws, stream=stream)
        if st != 0:
            return [self.fg.FgltError(st, "fglt_raw", "the request's CSR breaks the contract")]
        return self._finish(stream, [out], [(off, idx)])

    def run_batch(self, reqs, stream):
        torch = self.torch
        fg = self.fg
        vtx, off, idx = fg.batch_pack([(r.offsets, r.indices) for r in reqs])
        L = fg._lib.lib()
        G, n_total, nnz = len(reqs), int(vtx[-1]), int(idx.numel())
        with torch.cuda.stream(stream):
            off_d = off.to(self.device, non_blocking=True)
            idx_d = idx.to(self.device, non_blocking=True)
            ws = torch.empty(max(int(L.fglt_batch_workspace(G, n_total, nnz)), 1), dtype=torch.uint8,
                             device=self.device)
            out = fg.batch(vtx, off_d, idx_d, plan=self.batch_plan, workspace=ws, stream=stream)
            status = fg.batch_status(ws, stream=stream)
        if status != 0:
            # a request broke the contract: its rows were skipped on the device;
            # run the requests one at a time so that only the bad one fails
            return [self.run_single(r, stream)[0] for r in reqs]
        b = vtx.tolist()
        nets = [out[b[k]:b[k + 1]] for k in range(G)]
        e = off.tolist()
        csrs = [(off_d[b[k]:b[k + 1] + 1], idx_d[e[b[k]]:e[b[k + 1]]]) for k in range(G)]
        return self._finish(stream, nets, csrs, [(b[k], e[b[k]]) for k in range(G)])


class Server:
    def __init__(self, executor, budget_bytes: int = 64 << 30, streams: int = 4, small_n: int = 512,
                 max_batch: int = 4096):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.free = int(budget_bytes)
        self.small_n = small_n
        self.max_batch = max_batch
        self._ids = itertools.count()
        self._cv = threading.Condition()
        self._queue: list[Request] = []
        self._resident: dict[int, int] = {}
        self._running = 0
        self._stop = False
        self.latencies: list[float] = []
        self.completed = 0
        self._workers = [threading.Thread(target=self._work, args=(executor.make_stream(),),
                                          name=f"fglt-worker-{k}", daemon=True) for k in range(streams)]
        for t in self._workers:
            t.start()

    # ------------------------------------------------------------------ client API
    def submit(self, offsets, indices) -> Future:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        req = Request(next(self._ids), off, idx, time.perf_counter())
        req.future.rid = req.rid
        req.future.cancel_request = lambda r=req: self._cancel(r)
        try:
            from paper_2007_11111_amd import check_host_csr
        except Exception:  # the package without its library still offers the check
            check_host_csr = None
        if check_host_csr is not None:
            try:
                check_host_csr(off, idx)
            except ValueError as e:
                req.future.set_exception(e)
                return req.future
        small = req.n <= self.small_n
        req.bytes_resident, req.bytes_work = self.ex.bytes_for(req.n, req.nnz, small)
        if req.bytes_resident + req.bytes_work > self.budget:
            req.future.set_exception(Rejected(f"request {req.rid} needs "
                                              f"{req.bytes_resident + req.bytes_work} bytes > budget {self.budget}"))
            return req.future
        with self._cv:
            self._queue.append(req)
            self._cv.notify_all()
        return req.future

    def close(self, wait=True):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        if wait:
            for t in self._workers:
                t.join()

    @property
    def num_workers(self):
        return len(self._workers)

    def stats(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"completed": self.completed, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99)), "free_bytes": self.free}

    # ------------------------------------------------------------------ internals
    def _cancel(self, req):
        with self._cv:
            if req in self._queue:
                self._queue.remove(req)
                req.future.set_exception(Cancelled(f"request {req.rid} cancelled"))
                self._cv.notify_all()
                return True
        return False

    def _release(self, rid):
        with self._cv:
            b = self._resident.pop(rid, 0)
            self.free += b
            self._cv.notify_all()

    def _pick(self):
        """Next launch: (list of requests, is_batch), or None.  Arrival order with
        skip-ahead: a request that does not fit the free budget yet is passed over."""
        free = self.free
        picked = []
        small_mode = None
        for req in self._queue:
            need = req.bytes_resident + req.bytes_work
            if need > free:
                continue
            small = req.n <= self.small_n
            if small_mode is None:
                small_mode = small
            if small != small_mode:
                continue
            picked.append(req)
            free -= need
            if not small or len(picked) >= self.max_batch:
                break
        if not picked:
            return None
        return picked, bool(small_mode)

    def _work(self, stream):
        while True:
            with self._cv:
                while True:
                    if self._stop and not self._queue:
                        return
                    choice = self._pick() if self._queue else None
                    if choice is not None:
                        break
                    self._cv.wait(timeout=0.05)
                reqs, is_batch = choice
                for r in reqs:
                    self._queue.remove(r)
                    self.free -= r.bytes_resident + r.bytes_work
                    r.start = time.perf_counter()
                self._running += 1
            self._run(reqs, is_batch, stream)

    def _run(self, reqs, is_batch, stream):
        err = None
        outs = None
        try:
            outs = self.ex.run_batch(reqs, stream) if is_batch else self.ex.run_single(reqs[0], stream)
        except Exception as e:  # the executor failed: fail these requests, keep serving
            err = e
        end = time.perf_counter()
        with self._cv:
            for k, r in enumerate(reqs):
                r.end = end
                self.free += r.bytes_work
                o = err if err is not None else outs[k]
                if isinstance(o, Exception):
                    self.free += r.bytes_resident
                    r.future.set_exception(o)
                    continue
                self._resident[r.rid] = r.bytes_resident
                if isinstance(o, Outcome):
                    t_done = o.t_done or end
                    res = Result(r.rid, o.net, t_done - r.arrival, r.start - r.arrival, len(reqs),
                                 (o.t_host - r.arrival) if o.t_host else 0.0, o.csr, o.host_net, self,
                                 o.csr_base)
                else:
                    res = Result(r.rid, o, end - r.arrival, r.start - r.arrival, len(reqs), _server=self)
                self.latencies.append(res.latency_s)
                self.completed += 1
                r.future.set_result(res)
            self._running -= 1
            self._cv.notify_all()
