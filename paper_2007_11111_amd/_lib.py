"""ctypes loader for libfglt.so (the HIP library built by build.py).

There is no fallback: if the shared library is missing or fails to load, every
entry point raises.  Build it with ``python -m paper_2007_11111_amd.build``.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfglt.so")

NORBITS = 16
FGLT_NET = 1

STATUS = {
    0: "FGLT_OK",
    -1: "FGLT_EINVAL",
    -2: "FGLT_ENOTCANON",
    -3: "FGLT_EWORKSPACE",
    -4: "FGLT_EOVERFLOW",
    -5: "FGLT_EHIP",
    -6: "FGLT_EUNSUPPORTED",
}


class FgltError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({message})")


FGLT_TIMING = 2
FGLT_WORKMODEL = 8
FGLT_VALIDATE = 16
FGLT_PROGRESS = 32


def FGLT_SIGMA(mask: int) -> int:
    """Flag bits of a sub-dictionary with index set `mask` (bit k = orbit k)."""
    return (int(mask) & 0xFFFF) << 16


FGLT_SIGMA5 = FGLT_SIGMA(0x1F)
SEGMENTS = ["check", "relabel", "structure", "tri1_wave", "tri1_lds", "tri1_global", "fill",
            "tri2_wave", "tri2_lds", "tri2_global", "l2", "c4_wave", "c4_block", "c4_hash", "c4_window",
            "finalize"]


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "nnz", "d_max", "dplus_max", "tri_items", "wedge_items")] + [
        ("tri_tier_vertices", ctypes.c_int64 * 3), ("c4_tier_vertices", ctypes.c_int64 * 4),
        ("tri_items_tier", ctypes.c_int64 * 3), ("wedge_items_tier", ctypes.c_int64 * 4),
        ("triangles", ctypes.c_int64), ("min_sum", ctypes.c_int64), ("k4_merge", ctypes.c_int64),
        ("seg_ms", ctypes.c_float * len(SEGMENTS))]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name == "seg_ms":
                d[name] = {SEGMENTS[k]: float(v[k]) for k in range(len(SEGMENTS))}
            elif name.endswith(("_tier", "_vertices")):
                d[name] = [int(x) for x in v]
            else:
                d[name] = int(v)
        return d


class RawPlan(ctypes.Structure):
    _fields_ = [("tri_wave_max", ctypes.c_int32), ("tri_lds_max", ctypes.c_int32),
                ("c4_wave_max", ctypes.c_int32), ("c4_block_max", ctypes.c_int32),
                ("c4_hash_max", ctypes.c_int32), ("c4_window_rows", ctypes.c_int32),
                ("tri_hub_max", ctypes.c_int32), ("c4_window_group", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("hub_degree", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: the HIP library must be built "
                    "(python -m paper_2007_11111_amd.build); there is no CPU fallback")
            L = ctypes.CDLL(LIB_PATH)
            i64, i32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
            L.fglt_build_csr_workspace.argtypes = [i64, i64]
            L.fglt_build_csr_workspace.restype = sz
            L.fglt_build_csr.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, sz, vp]
            L.fglt_build_csr.restype = ctypes.c_int
            L.fglt_raw_workspace.argtypes = [i64, i64]
            L.fglt_raw_workspace.restype = sz
            L.fglt_raw.argtypes = [i64, i64, vp, vp, vp, vp, sz, ctypes.c_uint, ctypes.POINTER(RawPlan),
                                   ctypes.POINTER(Stats), vp]
            L.fglt_raw.restype = ctypes.c_int
            L.fglt_raw_status.argtypes = [vp, vp]
            L.fglt_raw_status.restype = ctypes.c_int
            L.fglt_net.argtypes = [i64, vp, vp, vp]
            L.fglt_net.restype = ctypes.c_int
            L.fglt_totals.argtypes = [i64, vp, i64, vp, vp, vp]
            L.fglt_totals.restype = ctypes.c_int
            if hasattr(L, "fglt_batch"):
                L.fglt_batch_workspace.argtypes = [i32, i64, i64]
                L.fglt_batch_workspace.restype = sz
                L.fglt_batch.argtypes = [i32, vp, vp, i64, i64, vp, vp, vp, ctypes.POINTER(BatchPlan), vp, sz, vp]
                L.fglt_batch.restype = ctypes.c_int
                L.fglt_batch_tune.argtypes = [i32, vp, vp, i64, i64, vp, vp, vp, vp, sz, i32,
                                              ctypes.POINTER(BatchPlan), vp]
                L.fglt_batch_tune.restype = ctypes.c_int
                L.fglt_batch_status.argtypes = [vp, vp]
                L.fglt_batch_status.restype = ctypes.c_int
                L.fglt_batch_release.argtypes = [vp]
                L.fglt_batch_release.restype = ctypes.c_int
            L.fglt_status_string.argtypes = [ctypes.c_int]
            L.fglt_status_string.restype = ctypes.c_char_p
            L.fglt_version.argtypes = []
            L.fglt_version.restype = ctypes.c_int
            _lib = L
    return _lib


def check(status: int, where: str):
    if status != 0:
        msg = lib().fglt_status_string(status).decode()
        raise FgltError(status, where, msg)
