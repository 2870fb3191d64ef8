"""The C ABI library loads on the CPU and exports every declared entry point.

No compute calls are made here (there is no GPU); only the host-side argument
checks, which return before touching the device, are exercised.
"""
import ctypes
import os

import pytest

from tests._util import ROOT, header_functions

LIB = os.path.join(ROOT, "paper_2007_11111_amd", "libfglt.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2007_11111_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("fglt_build_csr", "fglt_raw", "fglt_net", "fglt_batch"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in header_functions() if not hasattr(lib, f)]
    assert not missing, f"not exported: {missing}"


def test_status_strings_and_version(lib):
    lib.fglt_status_string.restype = ctypes.c_char_p
    lib.fglt_status_string.argtypes = [ctypes.c_int]
    for code in range(0, -7, -1):
        s = lib.fglt_status_string(code)
        assert s and s != b"unknown status"
    assert lib.fglt_version() >= 1


def test_workspace_queries_are_host_only(lib):
    lib.fglt_raw_workspace.restype = ctypes.c_size_t
    lib.fglt_raw_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64]
    small = lib.fglt_raw_workspace(10, 20)
    big = lib.fglt_raw_workspace(1_000_000, 18_000_000)
    assert 0 < small < big
    assert lib.fglt_raw_workspace(-1, 0) == 0
    lib.fglt_build_csr_workspace.restype = ctypes.c_size_t
    lib.fglt_build_csr_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64]
    assert lib.fglt_build_csr_workspace(100, 1000) > 0


def test_host_argument_checks_need_no_device(lib):
    vp = ctypes.c_void_p
    lib.fglt_raw.restype = ctypes.c_int
    lib.fglt_raw.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_uint, vp, vp, vp]
    # negative sizes and n >= 2^31 are rejected before any HIP call
    assert lib.fglt_raw(-1, 0, None, None, None, None, 0, 0, None, None, None) == -1
    assert lib.fglt_raw(1 << 31, 0, None, None, None, None, 0, 0, None, None, None) == -1
    # NULL pointers with n > 0
    assert lib.fglt_raw(5, 8, None, None, None, None, 0, 0, None, None, None) == -1
    # unknown flag bits
    assert lib.fglt_raw(0, 0, None, None, None, None, 0, 0x80, None, None, None) == -1
    # the empty graph is a no-op, with every defined flag (FGLT_NET 1, FGLT_TIMING 2,
    # FGLT_WORKMODEL 8, FGLT_VALIDATE 16, FGLT_PROGRESS 32, sub-dictionary masks in
    # bits 16..31 that hold orbits 0 and 1)
    for flags in (0, 1, 2, 3, 8, 11, 16, 27, 32, 59, 0x1F << 16, (0x1F << 16) | 1, (0x8003 << 16) | 3,
                  0xFFFF << 16):
        assert lib.fglt_raw(0, 0, None, None, None, None, 0, flags, None, None, None) == 0
    for flags in (4, 64, 0x80, 0x1E << 16, 0x1D << 16, 0x8000 << 16):
        assert lib.fglt_raw(0, 0, None, None, None, None, 0, flags, None, None, None) == -1
    lib.fglt_net.restype = ctypes.c_int
    lib.fglt_net.argtypes = [ctypes.c_int64, vp, vp, vp]
    assert lib.fglt_net(-3, None, None, None) == -1
    assert lib.fglt_net(0, None, None, None) == 0
    lib.fglt_totals.restype = ctypes.c_int
    lib.fglt_totals.argtypes = [ctypes.c_int64, vp, ctypes.c_int64, vp, vp, vp]
    assert lib.fglt_totals(-1, None, 0, None, None, None) == -1
    assert lib.fglt_totals(0, None, 0, None, None, None) == 0
    assert lib.fglt_totals(2, None, 10, None, None, None) == -1


def test_binding_plan_matches_header():
    """The ctypes plan structure lists the header's fields in its order."""
    import re
    from paper_2007_11111_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "fglt.h")).read()
    body = re.search(r"typedef struct \{([^{}]*)\} fglt_raw_plan;", hdr).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"int32_t (\w+);", body)
    assert fields == [f for f, _ in _lib.RawPlan._fields_]


def test_binding_flags_match_header():
    import re
    from paper_2007_11111_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "fglt.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"#define FGLT_(NET|TIMING|WORKMODEL|VALIDATE|PROGRESS) (\d+)u", hdr)}
    assert defs == {"NET": _lib.FGLT_NET, "TIMING": _lib.FGLT_TIMING, "WORKMODEL": _lib.FGLT_WORKMODEL,
                    "VALIDATE": _lib.FGLT_VALIDATE, "PROGRESS": _lib.FGLT_PROGRESS}
    # the sub-dictionary field: FGLT_SIGMA(mask) puts the 16-bit mask in bits 16..31
    assert re.search(r"#define FGLT_SIGMA\(mask\) \(\(unsigned\)\(\(mask\) & 0xffffu\) << 16\)", hdr)
    assert re.search(r"#define FGLT_SIGMA5 FGLT_SIGMA\(0x001fu\)", hdr)
    assert _lib.FGLT_SIGMA(0x1F) == _lib.FGLT_SIGMA5 == 0x1F << 16
