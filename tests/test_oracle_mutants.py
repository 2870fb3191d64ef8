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


# The same for the Python parts of the oracle: the Sigma_5 route by sparse
# products and the graph-level totals.  A mutant is the function's source
# with one planted mistake, compiled into a copy of the oracle's namespace.
PY_MUTANTS = [
    ("sigma5", "p2 keeps the walk back", "p2 = A @ p1 - p1", "p2 = A @ p1"),
    ("sigma5", "c3 not halved", "c3 //= 2", "c3 //= 1"),
    ("sigma5", "c3 without the edge mask", "A.multiply(A @ A)", "(A @ A)"),
    ("sigma5", "C(p1, 2) shifted", "p1 * (p1 - 1) // 2", "p1 * (p1 + 1) // 2"),
    ("sigma5", "net d2 takes c3 once", "out[:, 2] -= 2 * c3", "out[:, 2] -= c3"),
    ("sigma5", "net d3 takes c3 twice", "out[:, 3] -= c3", "out[:, 3] -= 2 * c3"),
    ("totals", "no division by m_k", "out[g] = col // ORBIT_NODES", "out[g] = col"),
    ("totals", "every graph's rows", "col = f[off[g]:off[g + 1]].sum(axis=0)", "col = f.sum(axis=0)"),
    ("subdict", "sign flipped", "out[:, a] -= u[a, b] * out[:, b]", "out[:, a] += u[a, b] * out[:, b]"),
    ("subdict", "forward order", "for a in range(len(s) - 1, -1, -1):", "for a in range(len(s)):"),
    ("subdict", "transposed block", "u = U16()[np.ix_(s, s)]", "u = U16().T[np.ix_(s, s)]"),
    ("subdict", "raw-only output converted", "if not net:", "if net is None:"),
    ("subdict", "inner loop misses the last orbit", "for b in range(a + 1, len(s)):",
     "for b in range(a + 1, len(s) - 1):"),
]


def _mutated(fn, old, new):
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(getattr(oracle, fn)))
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    ns = dict(vars(oracle))
    exec(compile(src.replace(old, new), f"<mutant of oracle.{fn}>", "exec"), ns)
    return ns[fn]


def _edges_of(n, off, idx):
    return [(i, int(j)) for i in range(n) for j in idx[off[i]:off[i + 1]] if i < j]


def _sigma5_ok(f):
    for n, off, idx, (br, bn) in _CASES:
        try:
            if not (np.array_equal(f(off, idx), br[:, :5]) and np.array_equal(f(off, idx, net=True), bn[:, :5])):
                return False
        except Exception:
            return False
    return True


def _totals_ok(f):
    # each case alone, then the first two cases as one batch of two graphs
    for n, off, idx, (_, bn) in _CASES:
        try:
            if not np.array_equal(f(bn)[0], bruteforce.graphlet_copies(n, _edges_of(n, off, idx))):
                return False
        except Exception:
            return False
    (n1, o1, i1, (_, b1)), (n2, o2, i2, (_, b2)) = _CASES[0], _CASES[1]
    exp = np.stack([bruteforce.graphlet_copies(n1, _edges_of(n1, o1, i1)),
                    bruteforce.graphlet_copies(n2, _edges_of(n2, o2, i2))])
    try:
        return np.array_equal(f(np.concatenate([b1, b2]), [0, n1, n1 + n2]), exp)
    except Exception:
        return False


def _subdict_ok(f):
    from tests.test_oracle_pins import CLOSED, OPEN, _relative_net
    u = oracle.U16()
    for n, off, idx, (br, bn) in _CASES:
        r = oracle.raw(off, idx)
        for s in CLOSED + OPEN:
            try:
                if not np.array_equal(f(r, s, net=False), br[:, s]):
                    return False
                if not np.array_equal(f(r, s), bn[:, s] if s in CLOSED else _relative_net(bn, s, u)):
                    return False
            except Exception:
                return False
    return True


def test_python_pins_accept_the_oracle():
    global _CASES
    if _CASES is None:
        _CASES = _cases()
    assert _sigma5_ok(oracle.sigma5) and _totals_ok(oracle.totals) and _subdict_ok(oracle.subdict)


@pytest.mark.parametrize("fn,name,old,new", PY_MUTANTS, ids=[f"{m[0]}: {m[1]}" for m in PY_MUTANTS])
def test_python_mutant_is_caught(fn, name, old, new):
    global _CASES
    if _CASES is None:
        _CASES = _cases()
    f = _mutated(fn, old, new)
    ok = {"sigma5": _sigma5_ok, "totals": _totals_ok, "subdict": _subdict_ok}[fn](f)
    assert not ok, f"mutant '{name}' of oracle.{fn} survived every pin"
