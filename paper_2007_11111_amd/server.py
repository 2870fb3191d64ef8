"""Serving runtime: continuous batching of graphlet-transform requests.

A request is one graph (host CSR).  The server
  * admits requests by an HBM budget: the bytes a request holds on the device
    (its CSR, its n x 16 result, and -- while it runs -- its workspace) must
    fit the free budget; a request larger than the whole budget is rejected;
  * keeps admitted CSRs and results resident on the device until the client
    releases them (the budget is returned then);
  * batches continuously: whenever a worker stream frees up, the scheduler
    takes the waiting requests in arrival order (skipping ahead past a request
    that does not fit yet) and either packs the small graphs (n <= small_n)
    into one fglt_batch launch or hands one large graph to fglt_raw; several
    worker streams run at once, so their work overlaps on the GPU;
  * records per-request latency from arrival to the completion of its kernels.

The device work goes through an executor object; ``GpuExecutor`` calls the HIP
library.  Tests substitute a CPU executor to drive the scheduling logic
without a GPU.
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
    cancelled: bool = False
    start: float = 0.0
    end: float = 0.0
    device_result: object = None

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])


@dataclass
class Result:
    rid: int
    net: object              # device tensor (GpuExecutor) or ndarray; n x 16 int64
    latency_s: float
    queued_s: float
    batched_with: int        # number of requests in the same launch
    _server: "Server" = None

    def release(self):
        """Returns the request's resident bytes to the budget."""
        if self._server is not None:
            self._server._release(self.rid)
            self._server = None


class GpuExecutor:
    """Runs requests on the GPU through the C ABI (one HIP stream per worker)."""

    def __init__(self, device=0, batch_plan=None):
        import torch
        import paper_2007_11111_amd as fg
        self.torch = torch
        self.fg = fg
        self.device = torch.device("cuda", device)
        self.batch_plan = batch_plan

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

    def run_single(self, req, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            off = torch.from_numpy(req.offsets).to(self.device, non_blocking=False)
            idx = torch.from_numpy(req.indices).to(self.device, non_blocking=False)
            out = self.fg.transform(off, idx, stream=stream)
            stream.synchronize()
        return [out]

    def run_batch(self, reqs, stream):
        torch = self.torch
        vtx, off, idx = self.fg.batch_pack([(r.offsets, r.indices) for r in reqs])
        with torch.cuda.stream(stream):
            off_d = off.to(self.device)
            idx_d = idx.to(self.device)
            out = self.fg.batch(vtx, off_d, idx_d, plan=self.batch_plan, stream=stream)
            stream.synchronize()
        bounds = vtx.tolist()
        return [out[bounds[k]:bounds[k + 1]] for k in range(len(reqs))]


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
        self._idle_streams = [executor.make_stream() for _ in range(streams)]
        self._running = 0
        self._stop = False
        self.latencies: list[float] = []
        self.completed = 0
        self._sched = threading.Thread(target=self._loop, name="fglt-scheduler", daemon=True)
        self._sched.start()

    # ------------------------------------------------------------------ client API
    def submit(self, offsets, indices) -> Future:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        req = Request(next(self._ids), off, idx, time.perf_counter())
        small = req.n <= self.small_n
        req.bytes_resident, req.bytes_work = self.ex.bytes_for(req.n, req.nnz, small)
        req.future.rid = req.rid
        req.future.cancel_request = lambda r=req: self._cancel(r)
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
            self._sched.join()

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

    def _loop(self):
        while True:
            with self._cv:
                while True:
                    if self._stop and not self._queue and self._running == 0:
                        return
                    if self._idle_streams and self._queue:
                        choice = self._pick()
                        if choice is not None:
                            break
                    self._cv.wait(timeout=0.05)
                reqs, is_batch = choice
                for r in reqs:
                    self._queue.remove(r)
                    self.free -= r.bytes_resident + r.bytes_work
                    r.start = time.perf_counter()
                stream = self._idle_streams.pop()
                self._running += 1
            threading.Thread(target=self._run, args=(reqs, is_batch, stream), daemon=True).start()

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
                if err is not None:
                    self.free += r.bytes_resident
                    r.future.set_exception(err)
                    continue
                self._resident[r.rid] = r.bytes_resident
                lat = end - r.arrival
                self.latencies.append(lat)
                self.completed += 1
                r.future.set_result(Result(r.rid, outs[k], lat, r.start - r.arrival, len(reqs), self))
            self._idle_streams.append(stream)
            self._running -= 1
            self._cv.notify_all()
