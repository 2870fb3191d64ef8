"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, a transposed
operand, a wrong coefficient) in a temporary copy of the oracle's C source,
builds it on the CPU, and checks that the worked example of Fig. 2 or the
brute-force enumeration on small random graphs rejects it.
"""
import ctypes
import os
import subprocess
from itertools import combinations

import numpy as np
import pytest

import oracle
from oracle import bruteforce

SRC = os.path.join(os.path.dirname(oracle.__file__), "fglt_oracle.c")

MUTANTS = [
    ("p2 drops c2", "p2[j] = rdiff(ap1, p1[j]);", "p2[j] = ap1;"),
    ("p3 drops -2c3", "r[5] = rdiff(rdiff(ap2, p1[i] * rdiff(p1[i], 1)), 2 * c3[i]);",
     "r[5] = rdiff(ap2, p1[i] * rdiff(p1[i], 1));"),
    ("d6 halves 2c3", "r[6] = rdiff(p2[i] * rdiff(p1[i], 1), 2 * c3[i]);",
     "r[6] = rdiff(p2[i] * rdiff(p1[i], 1), c3[i]);"),
    ("d7 wrong factor", "a7 += rdiff(p1[j], 1) * rdiff(p1[j], 2);", "a7 += rdiff(p1[j], 1) * rdiff(p1[j], 1);"),
    ("d8 wrong factor", "r[8] = p1[i] * rdiff(p1[i], 1) * rdiff(p1[i], 2) / 6;",
     "r[8] = p1[i] * p1[i] * rdiff(p1[i], 2) / 6;"),
    ("d9 halves 2c3", "r[9] = rdiff(ac3, 2 * c3[i]);", "r[9] = rdiff(ac3, c3[i]);"),
    ("d10 transposed operand", "c3p += C3[q] * rdiff(p1[j], 2);", "c3p += C3[q] * rdiff(p1[i], 2);"),
    ("d11 wrong shift", "r[11] = rdiff(p1[i], 2) * c3[i];", "r[11] = rdiff(p1[i], 1) * c3[i];"),
    ("c4 keeps k == i", "if (k == i) continue;", ""),
    ("d13 drops -A", "d4c += rdiff(C3[t], 1);", "d4c += C3[t];"),
    ("d14 drops -1", "d43 += v * rdiff(v, 1);", "d43 += v * v;"),
    ("d15 divides by 3", "r[15] = te / 6;", "r[15] = te / 3;"),
    ("U16(5,13) wrong", "{5, 13, 4}", "{5, 13, 2}"),
    ("U16(12,15) wrong", "{12, 15, 3}", "{12, 15, 1}"),
    ("back-substitution sign", "s -= u[k * NORB + c] * f[c];", "s += u[k * NORB + c] * f[c];"),
    ("C3 off by one", "C3[q] = cnt;", "C3[q] = cnt + 1;"),
]


def _cases():
    rng = np.random.default_rng(99)
    cases = [(6, [(5, 3), (3, 4), (4, 0), (0, 1), (1, 4), (1, 2), (2, 3), (2, 4), (1, 3)])]
    for _ in range(12):
        n = int(rng.integers(5, 9))
        edges = [(i, j) for i, j in combinations(range(n), 2) if rng.random() < 0.55]
        cases.append((n, edges))
    out = []
    for n, edges in cases:
        off, idx = oracle.canonical_csr(n, np.array([a for a, _ in edges], dtype=np.int64),
                                        np.array([b for _, b in edges], dtype=np.int64))
        out.append((n, off, idx, bruteforce.frequencies(n, edges)))
    return out


_CASES = None


def _net_with(lib, off, idx):
    n = off.shape[0] - 1
    p64 = ctypes.POINTER(ctypes.c_int64)
    p32 = ctypes.POINTER(ctypes.c_int32)
    raw = np.zeros((n, 16), dtype=np.int64)
    net = np.zeros((n, 16), dtype=np.int64)
    idx = np.ascontiguousarray(idx if idx.size else np.zeros(1, np.int32), dtype=np.int32)
    st = lib.oracle_raw(ctypes.c_int64(n), off.ctypes.data_as(p64), idx.ctypes.data_as(p32),
                        ctypes.c_int64(n), p64(), raw.ctypes.data_as(p64), ctypes.c_int(1))
    if st != 0:
        return None, None
    lib.oracle_raw_to_net(ctypes.c_int64(n), raw.ctypes.data_as(p64), net.ctypes.data_as(p64))
    return raw, net


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    global _CASES
    if _CASES is None:
        _CASES = _cases()
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-std=c11", "-w", "-o", str(so), str(mutated)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    lib.oracle_raw.restype = ctypes.c_int
    caught = False
    for n, off, idx, (br, bn) in _CASES:
        raw, net = _net_with(lib, off, idx)
        if raw is None or not (np.array_equal(raw, br) and np.array_equal(net, bn)):
            caught = True
            break
    assert caught, f"mutant '{name}' survived every pin"
