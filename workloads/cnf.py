"""Seeded CNF generators and the plain CNF container used as input data.

CNF layout (shared by every consumer as plain arrays): variables are
``1..n_vars``; ``lits`` holds DIMACS literals (``+v`` / ``-v``); clause ``c``
is ``lits[clause_off[c]:clause_off[c+1]]``.  No clause repeats a variable.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CNF:
    n_vars: int
    clause_off: np.ndarray   # uint64 [n_clauses + 1]
    lits: np.ndarray         # int32  [n_lits]
    name: str = ""

    @property
    def n_clauses(self) -> int:
        return len(self.clause_off) - 1

    def clauses(self):
        off, lits = self.clause_off, self.lits
        return [lits[off[c]:off[c + 1]].tolist() for c in range(self.n_clauses)]

    @staticmethod
    def from_clauses(n_vars: int, clauses, name: str = "") -> "CNF":
        off = np.zeros(len(clauses) + 1, dtype=np.uint64)
        flat = []
        for i, c in enumerate(clauses):
            assert len({abs(x) for x in c}) == len(c), "repeated variable"
            assert all(1 <= abs(x) <= n_vars for x in c)
            flat.extend(int(x) for x in c)
            off[i + 1] = len(flat)
        return CNF(n_vars, off, np.array(flat, dtype=np.int32), name)


def random_ksat(n: int, m: int, k: int, rng: np.random.Generator,
                name: str = "") -> CNF:
    """Uniform random k-SAT: every clause draws k distinct variables
    uniformly and independent uniform signs; clauses are independent."""
    vs = np.empty((m, k), dtype=np.int64)
    for c in range(m):
        vs[c] = rng.choice(n, size=k, replace=False) + 1
    signs = rng.integers(0, 2, size=(m, k)) * 2 - 1
    lits = (vs * signs).astype(np.int32).ravel()
    off = np.arange(0, m * k + 1, k, dtype=np.uint64)
    return CNF(n, off, lits, name or f"r{k}sat_n{n}_m{m}")


def random_3sat_threshold(n: int, rng: np.random.Generator,
                          ratio: float = 4.26) -> CNF:
    return random_ksat(n, int(round(ratio * n)), 3, rng)


def pigeonhole(pigeons: int, holes: int) -> CNF:
    """Pigeons into holes: every pigeon sits in some hole and no hole holds
    two pigeons.  Variable ``i*holes + j + 1`` means pigeon i is in hole j."""
    def x(i, j):
        return i * holes + j + 1
    clauses = [[x(i, j) for j in range(holes)] for i in range(pigeons)]
    for j in range(holes):
        for i in range(pigeons):
            for i2 in range(i + 1, pigeons):
                clauses.append([-x(i, j), -x(i2, j)])
    return CNF.from_clauses(pigeons * holes, clauses, f"php_{pigeons}_{holes}")


def concat(cnfs):
    """Batch arrays for several CNFs: (n_vars[nq], q_clause_start[nq+1],
    clause_off[C+1], lits[L]); clause offsets index the joined ``lits``."""
    n_vars = np.array([c.n_vars for c in cnfs], dtype=np.uint32)
    q_start = np.zeros(len(cnfs) + 1, dtype=np.uint64)
    offs, lits = [np.zeros(1, dtype=np.uint64)], []
    base_lit = 0
    for i, c in enumerate(cnfs):
        q_start[i + 1] = q_start[i] + c.n_clauses
        offs.append(c.clause_off[1:].astype(np.uint64) + np.uint64(base_lit))
        lits.append(c.lits.astype(np.int32))
        base_lit += len(c.lits)
    return (n_vars, q_start, np.concatenate(offs),
            np.concatenate(lits) if lits else np.zeros(0, np.int32))


def random_ksat_batch(n: int, m: int, k: int, count: int, rng: np.random.Generator,
                      prefix: str = "") -> list:
    """`count` independent uniform random k-SAT instances (the model of
    random_ksat), drawn with whole-array operations: each clause's k
    variables are uniform integers, rows with a repeated variable are drawn
    again until every row is distinct (rejection keeps the distribution
    uniform over distinct k-tuples)."""
    vs = rng.integers(1, n + 1, size=(count, m, k))
    while True:
        s = np.sort(vs, axis=2)
        bad = (s[:, :, 1:] == s[:, :, :-1]).any(axis=2)
        nb = int(bad.sum())
        if nb == 0:
            break
        vs[bad] = rng.integers(1, n + 1, size=(nb, k))
    signs = rng.integers(0, 2, size=(count, m, k)) * 2 - 1
    off = np.arange(0, m * k + 1, k, dtype=np.uint64)
    return [CNF(n, off, (vs[i] * signs[i]).astype(np.int32).ravel(),
                f"{prefix}r{k}sat_n{n}_m{m}_{i}") for i in range(count)]
