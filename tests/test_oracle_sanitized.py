"""The oracle's C code under the host sanitizers (ASan and UBSan), on the CPU.

A small driver (tests/oracle_sanitized_driver.c) is built with the oracle's
source and -fsanitize=address,undefined; it canonicalises raw pairs and
evaluates every vertex.  The run must end cleanly (any sanitizer report makes
it fail) and give the regular build's CSR and net counts bit for bit.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen
import oracle
from tests._util import ROOT

SRC = os.path.join(ROOT, "oracle", "fglt_oracle.c")
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitized_driver.c")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-o", exe, DRIVER, SRC]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _run(exe, tmp, n, src, dst):
    fin, fout = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
    with open(fin, "wb") as fh:
        np.array([n, src.size], dtype=np.int64).tofile(fh)
        src.astype(np.int32).tofile(fh)
        dst.astype(np.int32).tofile(fh)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    res = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-2000:]
    with open(fout, "rb") as fh:
        nnz = int(np.fromfile(fh, dtype=np.int64, count=1)[0])
        off = np.fromfile(fh, dtype=np.int64, count=n + 1)
        idx = np.fromfile(fh, dtype=np.int32, count=nnz)
        net = np.fromfile(fh, dtype=np.int64, count=n * 16).reshape(n, 16)
    return off, idx, net


@pytest.mark.parametrize("which", ["fig-sized", "er", "chung-lu", "clique", "empty"])
def test_oracle_under_sanitizers(sanitized, tmp_path, which):
    if which == "fig-sized":
        n, src, dst = 6, np.array([0, 0, 1, 1, 2, 3, 4, 4, 5, 2]), np.array([1, 2, 2, 3, 3, 4, 5, 2, 0, 2])
    elif which == "empty":
        n, src, dst = 5, np.zeros(0, np.int64), np.zeros(0, np.int64)
    else:
        g = {"er": lambda: graphgen.erdos_renyi(300, 0.05, seed=3),
             "chung-lu": lambda: graphgen.chung_lu(2000, 2.1, 10.0, 300.0, seed=4),
             "clique": lambda: graphgen.clique(24)}[which]()
        n, src, dst = g.n, g.src, g.dst
    off, idx, net = _run(sanitized, str(tmp_path), n, np.asarray(src), np.asarray(dst))
    off_r, idx_r = oracle.canonical_csr(n, src, dst)
    np.testing.assert_array_equal(off, off_r)
    np.testing.assert_array_equal(idx, idx_r)
    np.testing.assert_array_equal(net, oracle.net(off_r, idx_r))
