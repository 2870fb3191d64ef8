"""Fast graphlet transform on MI355X (gfx950).

Thin Python binding over the C ABI of ``libfglt.so`` (include/fglt.h): it only
allocates device buffers with torch, picks the current HIP stream and passes
raw pointers.  Every step of the transform runs in the library's HIP kernels.

    offsets, indices = build_csr(n, src, dst)          # canonical CSR on the GPU
    f = transform(offsets, indices)                    # n x 16 int64 net frequencies
    r = raw(offsets, indices); f = net(r)              # the two stages separately
    outs = batch([...])                                # many small graphs, one launch
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import FGLT_NET, FGLT_PROGRESS, FGLT_SIGMA, FGLT_TIMING, FGLT_VALIDATE, FGLT_WORKMODEL, NORBITS, SEGMENTS, BatchPlan, FgltError, RawPlan, Stats, check, lib

__all__ = [
    "build_csr", "raw", "raw_status", "net", "transform", "raw_workspace_bytes", "sigma_mask", "FgltError", "Stats",
    "BatchPlan", "check_host_csr", "batch_pack", "batch", "batch_tune", "batch_release", "batch_status", "totals", "NORBITS",
]


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(device=None):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


def build_csr(n: int, src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Canonical CSR (symmetric, no self-loops, no duplicates, sorted rows) of
    the undirected graph spanned by the pairs (src, dst) -- ``fglt_build_csr``.

    src, dst: int32 device tensors.  Returns (offsets int64[n+1], indices
    int32[nnz]) on the same device."""
    L = lib()
    assert src.dtype == torch.int32 and dst.dtype == torch.int32 and src.is_cuda and dst.is_cuda
    src = src.contiguous()
    dst = dst.contiguous()
    E = int(src.numel())
    dev = src.device
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    indices = torch.empty(max(2 * E, 1), dtype=torch.int32, device=dev)
    nnz = torch.empty(1, dtype=torch.int64, device=dev)
    ws_bytes = int(L.fglt_build_csr_workspace(n, E))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    check(L.fglt_build_csr(n, E, _ptr(src), _ptr(dst), _ptr(offsets), _ptr(indices), _ptr(nnz),
                           _ptr(ws), ws_bytes, _stream(stream)), "fglt_build_csr")
    m = int(nnz.item())
    if m < 0:
        raise FgltError(-1, "fglt_build_csr", "an endpoint is outside [0, n)")
    return offsets, indices[:m]


def sigma_mask(sigma) -> int:
    """16-bit orbit mask of a sub-dictionary (0: all 16 orbits) from None, an
    int mask, or an iterable of orbit numbers."""
    if sigma is None:
        return 0
    if isinstance(sigma, int):
        mask = sigma
    else:
        mask = 0
        for k in sigma:
            if not 0 <= int(k) < NORBITS:
                raise ValueError(f"orbit {k} is outside 0..15")
            mask |= 1 << int(k)
    if not 0 < mask <= 0xFFFF or mask & 3 != 3:
        raise ValueError(f"a sub-dictionary mask must hold orbits 0 and 1 and fit 16 bits: {mask:#x}")
    return 0 if mask == 0xFFFF else mask


def raw_workspace_bytes(n: int, nnz: int) -> int:
    return int(lib().fglt_raw_workspace(int(n), int(nnz)))


def raw(offsets: torch.Tensor, indices: torch.Tensor, *, net: bool = False, out: torch.Tensor | None = None,
        workspace: torch.Tensor | None = None, stats: bool = False, plan: dict | None = None,
        timing: bool = False, sigma=None, sigma5: bool = False, workmodel: bool = False, validate: bool = True,
        progress: bool = False, stream=None):
    """Raw frequencies (Table I) per vertex -- ``fglt_raw``; with net=True the
    net frequencies (Table I then Table II).  Returns an int64 [n, 16] tensor
    (and a dict of plan statistics when stats=True).  ``sigma`` selects a
    sub-dictionary (Section V): a 16-bit mask or an iterable of orbit numbers
    that holds 0 and 1; the result is then [n, |s|], the orbits of s in
    ascending order, net by U16(s, s).  sigma5=True is sigma=0x1F (Theorem 1).
    With validate=True (the default) the call waits for the stream and raises
    FgltError for a CSR that breaks the contract; validate=False enqueues the
    transform and returns at once (nothing waits: ``raw_status(workspace)``
    reads the device status word later; capturable into a HIP graph).  ``plan`` may set the tier
    thresholds tri_wave_max, tri_lds_max, tri_hub_max, c4_wave_max, c4_block_max, c4_hash_max, the
    window tier's row cuts c4_window_rows (0 default, 1 per-vertex table, 2 searches) and its
    windows per many-middle job c4_window_group (0 default, k exactly k); with
    timing=True the statistics carry per-segment milliseconds (HIP events); with
    workmodel=True (and stats=True) they carry the byte model's work terms
    min_sum and k4_merge (a statistics pass after the transform); with
    progress=True each launch segment's end is printed on stderr as the stream
    reaches it."""
    L = lib()
    assert offsets.dtype == torch.int64 and indices.dtype == torch.int32
    assert offsets.is_cuda and indices.is_cuda
    offsets = offsets.contiguous()
    indices = indices.contiguous()
    n = int(offsets.numel()) - 1
    nnz = int(indices.numel())
    dev = offsets.device
    mask = sigma_mask(0x1F if sigma5 else sigma)
    cols = bin(mask).count("1") if mask else NORBITS
    if out is None:
        out = torch.empty((max(n, 0), cols), dtype=torch.int64, device=dev)
    if out.dtype != torch.int64 or not out.is_contiguous() or out.device != dev or tuple(out.shape) != (max(n, 0), cols):
        raise ValueError(f"out must be a contiguous int64 tensor of shape ({n}, {cols}) on {dev}")
    ws_bytes = int(L.fglt_raw_workspace(n, nnz))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    st = Stats()
    rp = None
    if plan:
        rp = RawPlan(int(plan.get("tri_wave_max", 0)), int(plan.get("tri_lds_max", 0)),
                     int(plan.get("c4_wave_max", 0)), int(plan.get("c4_block_max", 0)),
                     int(plan.get("c4_hash_max", 0)), int(plan.get("c4_window_rows", 0)),
                     int(plan.get("tri_hub_max", 0)), int(plan.get("c4_window_group", 0)))
    check(L.fglt_raw(n, nnz, _ptr(offsets), _ptr(indices if nnz else None), _ptr(out), _ptr(workspace),
                     int(workspace.numel()), (FGLT_NET if net else 0) | (FGLT_TIMING if timing else 0) | FGLT_SIGMA(mask)
                     | (FGLT_VALIDATE if validate else 0)
                     | (FGLT_WORKMODEL if workmodel else 0) | (FGLT_PROGRESS if progress else 0),
                     ctypes.byref(rp) if rp is not None else None,
                     ctypes.byref(st) if stats else None, _stream(stream)),
          "fglt_raw")
    return (out, st.as_dict()) if stats else out


def raw_status(workspace: torch.Tensor, stream=None) -> int:
    """Status word of the last ``fglt_raw`` on `workspace` -- ``fglt_raw_status``
    (synchronizes with the stream): 0, FGLT_ENOTCANON (-2) or FGLT_EOVERFLOW (-4)."""
    return int(lib().fglt_raw_status(_ptr(workspace), _stream(stream)))


def net(raw_counts: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Net from raw frequencies, f = U16^{-1} raw per vertex -- ``fglt_net``."""
    L = lib()
    assert raw_counts.dtype == torch.int64 and raw_counts.is_cuda
    raw_counts = raw_counts.contiguous()
    n = int(raw_counts.shape[0])
    if out is None:
        out = torch.empty_like(raw_counts)
    check(L.fglt_net(n, _ptr(raw_counts), _ptr(out), _stream(stream)), "fglt_net")
    return out


def totals(net_counts: torch.Tensor, vtx_offsets: torch.Tensor | None = None, stream=None):
    """Graph-level totals -- ``fglt_totals``: for each graph (rows
    vtx_offsets[g] .. vtx_offsets[g+1]-1 of the net frequencies; one graph when
    vtx_offsets is None) and orbit k, the number of induced copies of orbit k's
    graphlet.  Returns an int64 [G, 16] tensor."""
    L = lib()
    assert net_counts.dtype == torch.int64 and net_counts.is_cuda
    net_counts = net_counts.contiguous()
    n = int(net_counts.shape[0])
    if vtx_offsets is None:
        vtx_offsets = torch.tensor([0, n], dtype=torch.int64, device=net_counts.device)
    assert vtx_offsets.dtype == torch.int64 and vtx_offsets.is_cuda
    vtx_offsets = vtx_offsets.contiguous()
    G = int(vtx_offsets.numel()) - 1
    out = torch.empty((max(G, 0), NORBITS), dtype=torch.int64, device=net_counts.device)
    check(L.fglt_totals(G, _ptr(vtx_offsets), n, _ptr(net_counts if n else None), _ptr(out), _stream(stream)),
          "fglt_totals")
    return out


def transform(offsets: torch.Tensor, indices: torch.Tensor, **kw):
    """Net frequencies of every vertex (the graphlet transform over Sigma_16)."""
    return raw(offsets, indices, net=True, **kw)


def check_host_csr(offsets, indices):
    """Structural checks of a host CSR before it is packed or sent to the
    device: offsets[0] == 0, offsets non-decreasing, offsets[-1] == len(indices).
    Raises ValueError.  (Symmetry, self-loops and repeated entries are checked
    on the device.)"""
    import numpy as np
    off = np.asarray(offsets)
    idx = np.asarray(indices)
    if off.ndim != 1 or off.shape[0] < 1:
        raise ValueError("offsets must be a 1-D array of n + 1 entries")
    if idx.ndim != 1:
        raise ValueError("indices must be a 1-D array")
    if int(off[0]) != 0:
        raise ValueError(f"offsets[0] is {int(off[0])}, not 0")
    if int(off[-1]) != idx.shape[0]:
        raise ValueError(f"offsets[-1] is {int(off[-1])}, not len(indices) = {idx.shape[0]}")
    if off.shape[0] > 1 and bool((np.diff(off) < 0).any()):
        raise ValueError("offsets decrease")


def batch_pack(csrs):
    """Block-diagonal packing of host CSRs [(offsets, indices), ...] (numpy or
    torch CPU) into (vtx_offsets, offsets, indices) int64/int64/int32 CPU
    tensors.  Each CSR must pass check_host_csr (ValueError otherwise)."""
    import numpy as np
    vtx = [0]
    offs = []
    idxs = []
    base_v = 0
    base_e = 0
    for off, idx in csrs:
        off = np.asarray(off, dtype=np.int64)
        idx = np.asarray(idx, dtype=np.int32)
        check_host_csr(off, idx)
        n = off.shape[0] - 1
        offs.append(off[:-1] + base_e)
        idxs.append(idx.astype(np.int64) + base_v)
        base_v += n
        base_e += int(off[-1])
        vtx.append(base_v)
    offs.append(np.array([base_e], dtype=np.int64))
    return (torch.from_numpy(np.array(vtx, dtype=np.int64)),
            torch.from_numpy(np.concatenate(offs)),
            torch.from_numpy(np.concatenate(idxs).astype(np.int32) if idxs else np.zeros(0, np.int32)))


def batch(vtx_offsets: torch.Tensor, offsets: torch.Tensor, indices: torch.Tensor, *, plan: dict | None = None,
          out: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None):
    """Net frequencies of many independent graphs in one fused launch --
    ``fglt_batch``.  vtx_offsets is a CPU int64 tensor [G+1]; offsets and
    indices are the block-diagonal CSR on the device."""
    L = lib()
    if not hasattr(L, "fglt_batch"):
        raise RuntimeError("libfglt.so was built without fglt_batch")
    vtx_host = vtx_offsets.to("cpu", torch.int64).contiguous()
    dev = offsets.device
    vtx_dev = vtx_host.to(dev)
    G = int(vtx_host.numel()) - 1
    n_total = int(vtx_host[-1])
    nnz = int(indices.numel())
    if out is None:
        out = torch.empty((n_total, NORBITS), dtype=torch.int64, device=dev)
    ws_bytes = int(L.fglt_batch_workspace(G, n_total, nnz))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    bp = None
    if plan is not None:
        bp = BatchPlan(int(plan.get("threads", 0)), int(plan.get("hub_degree", 0)),
                       int(plan.get("blocks_per_cu", 0)), int(plan.get("use_graph", 0)))
    check(L.fglt_batch(G, _ptr(vtx_dev), ctypes.c_void_p(vtx_host.data_ptr()), n_total, nnz, _ptr(offsets),
                       _ptr(indices if nnz else None), _ptr(out), ctypes.byref(bp) if bp is not None else None,
                       _ptr(workspace), int(workspace.numel()), _stream(stream)), "fglt_batch")
    return out


def batch_tune(vtx_offsets: torch.Tensor, offsets: torch.Tensor, indices: torch.Tensor, *, reps: int = 3,
               out: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None) -> dict:
    """Execution plan of ``fglt_batch`` for this batch -- ``fglt_batch_tune``
    (times the candidate plans, or returns the plan cached for the same batch
    shape and size histogram).  Returns the plan as a dict for ``batch``."""
    L = lib()
    vtx_host = vtx_offsets.to("cpu", torch.int64).contiguous()
    dev = offsets.device
    vtx_dev = vtx_host.to(dev)
    G = int(vtx_host.numel()) - 1
    n_total = int(vtx_host[-1])
    nnz = int(indices.numel())
    if out is None:
        out = torch.empty((n_total, NORBITS), dtype=torch.int64, device=dev)
    ws_bytes = int(L.fglt_batch_workspace(G, n_total, nnz))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    bp = BatchPlan()
    check(L.fglt_batch_tune(G, _ptr(vtx_dev), ctypes.c_void_p(vtx_host.data_ptr()), n_total, nnz, _ptr(offsets),
                            _ptr(indices if nnz else None), _ptr(out), _ptr(workspace), int(workspace.numel()),
                            int(reps), ctypes.byref(bp), _stream(stream)), "fglt_batch_tune")
    return {"threads": bp.threads, "hub_degree": bp.hub_degree, "blocks_per_cu": bp.blocks_per_cu,
            "use_graph": bp.use_graph}


def batch_release(stream=None):
    """Frees the HIP graphs ``fglt_batch`` cached for `stream` (None: all streams)."""
    L = lib()
    check(L.fglt_batch_release(ctypes.c_void_p(0 if stream is None else stream.cuda_stream)), "fglt_batch_release")


def batch_status(workspace: torch.Tensor, stream=None) -> int:
    """Status word of the last ``fglt_batch`` on `workspace` -- ``fglt_batch_status``
    (synchronizes with the stream): 0, or FGLT_ENOTCANON (-2) when a graph broke
    the contract and its rows were skipped."""
    return int(lib().fglt_batch_status(_ptr(workspace), _stream(stream)))
