"""ctypes front end of the plain C DPLL oracle (test infrastructure only).

Builds ``oracle/liboracle.so`` from ``dpll.c`` with gcc when it is missing
(``build()`` always rebuilds).  Also holds the numpy brute force that pins
the DPLL on tiny formulas.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpll.c")
LIB = os.path.join(HERE, "liboracle.so")

SAT, UNSAT, UNKNOWN = "SAT", "UNSAT", "UNKNOWN"
DEFAULT_NODES = 10_000_000

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                           "-Wall", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        L.oracle_solve.argtypes = [C.c_int32, C.c_int64, p, p, C.c_int64, p, p]
        L.oracle_solve.restype = C.c_int
        L.oracle_count.argtypes = [C.c_int32, C.c_int64, p, p, C.c_int64, p,
                                   C.c_int32, p]
        L.oracle_count.restype = C.c_int
        L.oracle_up.argtypes = [C.c_int32, C.c_int64, p, p, p, C.c_int32, p]
        L.oracle_up.restype = C.c_int
        L.oracle_leaf.argtypes = [C.c_int32, C.c_int64, p, p, p, C.c_int32,
                                  C.c_int64, p, p, p, p, C.c_int32, p, p]
        L.oracle_leaf.restype = C.c_int
        _lib = L
    return _lib


def _arrays(cnf):
    off = np.ascontiguousarray(cnf.clause_off, dtype=np.uint64)
    lits = np.ascontiguousarray(cnf.lits, dtype=np.int32)
    if len(lits) == 0:
        lits = np.zeros(1, dtype=np.int32)
    return off, lits


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def solve(cnf, max_nodes: int = DEFAULT_NODES):
    """DPLL decide: (verdict, model bytes [n+1] or None, nodes)."""
    off, lits = _arrays(cnf)
    model = np.zeros(cnf.n_vars + 1, dtype=np.uint8)
    nodes = C.c_int64(0)
    r = lib().oracle_solve(cnf.n_vars, cnf.n_clauses, _ptr(off), _ptr(lits),
                           max_nodes, _ptr(model), C.byref(nodes))
    verdict = {1: SAT, 0: UNSAT, 2: UNKNOWN}[r]
    return verdict, (model if r == 1 else None), nodes.value


def count(cnf, max_nodes: int = DEFAULT_NODES) -> int:
    """#DPLL model count over all variables (Python int); raises on budget."""
    off, lits = _arrays(cnf)
    words = cnf.n_vars // 32 + 2
    acc = np.zeros(words, dtype=np.uint32)
    r = lib().oracle_count(cnf.n_vars, cnf.n_clauses, _ptr(off), _ptr(lits),
                           max_nodes, _ptr(acc), words, None)
    if r != 0:
        raise RuntimeError(f"oracle_count failed ({r})")
    return sum(int(w) << (32 * i) for i, w in enumerate(acc))


def up(cnf, cube=()):
    """Unit-propagation fixpoint: (conflict, assign int8 [n+1], -1 = free)."""
    off, lits = _arrays(cnf)
    c = np.array(list(cube) or [0], dtype=np.int32)
    a = np.zeros(cnf.n_vars + 1, dtype=np.int8)
    r = lib().oracle_up(cnf.n_vars, cnf.n_clauses, _ptr(off), _ptr(lits),
                        _ptr(c), len(cube), _ptr(a))
    return bool(r), a


def leaf(cnf, cube=(), max_nodes: int = DEFAULT_NODES):
    """Canonical leaf of a cube: dict(refuted, f, m, slots, count, first)."""
    off, lits = _arrays(cnf)
    c = np.array(list(cube) or [0], dtype=np.int32)
    cap = 64
    slots = np.zeros(cap, dtype=np.int32)
    ref, f, m = C.c_int32(), C.c_int32(), C.c_int32()
    cnt, first = C.c_uint64(), C.c_int64()
    r = lib().oracle_leaf(cnf.n_vars, cnf.n_clauses, _ptr(off), _ptr(lits),
                          _ptr(c), len(cube), max_nodes, C.byref(ref),
                          C.byref(f), C.byref(m), _ptr(slots), cap,
                          C.byref(cnt), C.byref(first))
    if r == 2:
        raise RuntimeError("oracle_leaf: node budget exhausted")
    out = dict(refuted=bool(ref.value), f=f.value, m=m.value,
               slots=slots[:min(f.value, cap)].tolist(), count=None, first=None)
    if r == 0 and not ref.value:
        out["count"] = int(cnt.value)
        out["first"] = int(first.value)
    return out


# ------------------------------------------------------------ brute force

def brute_force(cnf):
    """All 2**n assignments (n <= 22): (number of models, sorted model
    indices as ints where bit v-1 is variable v)."""
    n = cnf.n_vars
    assert n <= 22
    idx = np.arange(1 << n, dtype=np.int64)
    ok = np.ones(1 << n, dtype=bool)
    for cl in cnf.clauses():
        sat = np.zeros(1 << n, dtype=bool)
        for l in cl:
            bit = (idx >> (abs(l) - 1)) & 1
            sat |= (bit == 1) if l > 0 else (bit == 0)
        ok &= sat
    models = idx[ok]
    return int(ok.sum()), models


def check_model(cnf, model) -> bool:
    """Every clause has a true literal under model (sequence indexed 1..n)."""
    for cl in cnf.clauses():
        if not any((model[abs(l)] == 1) == (l > 0) for l in cl):
            return False
    return True
