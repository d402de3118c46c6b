"""Exact-integer meaning of an OOB query: TEST INFRASTRUCTURE ONLY.

A query (Sec. 4.1 and Sec. 5.2 of the paper) is satisfiable iff some legal
input makes every constraint hold at once: ids below their dimensions
(kind 1), the offset reaching the size (kind 2), and the defining equalities
and asserts (kind 3).  SAT means the access can go out of bounds; UNSAT that
it cannot under any input.  Arithmetic is over the unbounded integers and
inputs range over ``0 .. 2**width - 1``.

Contents
* ``int_eval``        - the definition, written out with Python integers.
* ``int_bruteforce``  - every input tuple (<= 22 input bits), vectorised.
* ``encode``          - the oracle's own Tseitin encoding (two's complement,
  widths that never overflow, full-equivalence gates): an independent
  re-derivation of the CNF route, used to decide queries at full width.
* ``root_check``      - the oracle's word-level reasoning (the same method as
  the library's root stage, written apart from it; only its soundness is
  pinned, against exhaustive search): every comparison
  is brought to a polynomial normal form and the bounds asserted on the same
  polynomial are intersected; an empty intersection proves UNSAT.  Failing
  that, the root facts, their products with single atoms (kept when every
  monomial they produce already occurs in the facts) and the value range of
  every monomial form a linear system over the monomials; if it has no
  rational solution (Fourier-Motzkin elimination) the query is UNSAT.
* ``decide``          - root check, else encode + DPLL.
* ``wrap_eval`` / ``wrap_bruteforce`` - the same definition with m-bit
  machine integers (every integer node modulo 2**m, unsigned comparisons).
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import gcd

import numpy as np

from workloads.query import (OP_VAR, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_SHL,
                             OP_UDIV, OP_UREM, OP_LT, OP_LE, OP_GT, OP_GE,
                             OP_EQ, OP_NE, OP_AND, OP_OR, OP_NOT)
from workloads.cnf import CNF
from . import cnf_ref

SAT, UNSAT, UNKNOWN = "SAT", "UNSAT", "UNKNOWN"


def _nodes(q):
    return q.nodes, q.roots, q.var_widths


# ------------------------------------------------------------ definition

def int_eval_nodes(q, values):
    """Value of every node (int or bool) for the inputs ``values``
    (list indexed by declaration number)."""
    nodes, _, widths = _nodes(q)
    val = []
    for (op, a, b, w, imm) in nodes:
        if op == OP_VAR:
            x = int(values[imm])
            assert 0 <= x < (1 << widths[imm]), "input out of its domain"
            val.append(x)
        elif op == OP_CONST:
            val.append(int(imm))
        elif op == OP_ADD:
            val.append(val[a] + val[b])
        elif op == OP_SUB:
            val.append(val[a] - val[b])
        elif op == OP_MUL:
            val.append(val[a] * val[b])
        elif op == OP_SHL:
            val.append(val[a] * (1 << imm))
        elif op in (OP_UDIV, OP_UREM):
            assert val[a] >= 0, "division of a negative value"
            val.append(val[a] // imm if op == OP_UDIV else val[a] % imm)
        elif op == OP_LT:
            val.append(val[a] < val[b])
        elif op == OP_LE:
            val.append(val[a] <= val[b])
        elif op == OP_GT:
            val.append(val[a] > val[b])
        elif op == OP_GE:
            val.append(val[a] >= val[b])
        elif op == OP_EQ:
            val.append(val[a] == val[b])
        elif op == OP_NE:
            val.append(val[a] != val[b])
        elif op == OP_AND:
            val.append(bool(val[a]) and bool(val[b]))
        elif op == OP_OR:
            val.append(bool(val[a]) or bool(val[b]))
        elif op == OP_NOT:
            val.append(not bool(val[a]))
        else:
            raise ValueError(f"unknown op {op}")
    return val


def int_eval(q, values) -> bool:
    """True iff every root holds for the inputs (exact integers)."""
    val = int_eval_nodes(q, values)
    return all(bool(val[r]) for r in q.roots)


def int_eval_named(q, named: dict) -> bool:
    return int_eval(q, [named[n] for n in q.var_names])


# ---------------------------------------------------------------- machine integers
# The variant with m-bit machine integers (the semantics a 32-bit CUDA index
# computation has, where it can overflow): every integer node is reduced
# modulo 2**m, division and remainder are unsigned, comparisons compare the
# reduced values.  Written out from that definition, apart from the exact
# evaluator above.

def wrap_eval_nodes(q, values, m: int):
    """Value of every node with m-bit machine integers."""
    mod = 1 << m
    nodes, _, widths = _nodes(q)
    val = []
    for (op, a, b, w, imm) in nodes:
        if op == OP_VAR:
            x = int(values[imm])
            assert 0 <= x < (1 << widths[imm]), "input out of its domain"
            val.append(x % mod)
        elif op == OP_CONST:
            val.append(int(imm) % mod)
        elif op == OP_ADD:
            val.append((val[a] + val[b]) % mod)
        elif op == OP_SUB:
            val.append((val[a] - val[b]) % mod)
        elif op == OP_MUL:
            val.append((val[a] * val[b]) % mod)
        elif op == OP_SHL:
            val.append((val[a] << imm) % mod)
        elif op == OP_UDIV:
            val.append(val[a] // imm)
        elif op == OP_UREM:
            val.append(val[a] % imm)
        elif op == OP_LT:
            val.append(val[a] < val[b])
        elif op == OP_LE:
            val.append(val[a] <= val[b])
        elif op == OP_GT:
            val.append(val[a] > val[b])
        elif op == OP_GE:
            val.append(val[a] >= val[b])
        elif op == OP_EQ:
            val.append(val[a] == val[b])
        elif op == OP_NE:
            val.append(val[a] != val[b])
        elif op == OP_AND:
            val.append(bool(val[a]) and bool(val[b]))
        elif op == OP_OR:
            val.append(bool(val[a]) or bool(val[b]))
        elif op == OP_NOT:
            val.append(not bool(val[a]))
        else:
            raise ValueError(op)
    return val


def wrap_eval(q, values, m: int) -> bool:
    """True iff every root holds for the inputs with m-bit machine integers."""
    val = wrap_eval_nodes(q, values, m)
    return all(bool(val[r]) for r in q.roots)


def wrap_bruteforce(q, m: int, max_bits: int = 22):
    """Every input tuple (product order, first declared slowest) with m-bit
    machine integers; (verdict, number of satisfying tuples, first one)."""
    assert 1 <= m <= 63
    bits = sum(q.var_widths)
    assert bits <= max_bits, f"{bits} input bits is too many for brute force"
    grids = np.meshgrid(*[np.arange(1 << w, dtype=np.int64) for w in q.var_widths], indexing="ij")
    cols = [g.ravel() for g in grids]
    n = cols[0].size if cols else 1
    mod = 1 << m

    def red(x):   # Python-object arithmetic, then reduced: no int64 overflow
        return np.array([int(v) % mod for v in x], dtype=object) if x.dtype == object else x % mod

    val = []
    for (op, a, b, w, imm) in q.nodes:
        if op == OP_VAR:
            val.append(cols[imm].astype(object) % mod)
        elif op == OP_CONST:
            val.append(np.full(n, int(imm) % mod, dtype=object))
        elif op == OP_ADD:
            val.append(red(val[a] + val[b]))
        elif op == OP_SUB:
            val.append(red(val[a] - val[b]))
        elif op == OP_MUL:
            val.append(red(val[a] * val[b]))
        elif op == OP_SHL:
            val.append(red(val[a] * (1 << int(imm))))
        elif op == OP_UDIV:
            val.append(val[a] // int(imm))
        elif op == OP_UREM:
            val.append(val[a] % int(imm))
        elif op == OP_LT:
            val.append(val[a] < val[b])
        elif op == OP_LE:
            val.append(val[a] <= val[b])
        elif op == OP_GT:
            val.append(val[a] > val[b])
        elif op == OP_GE:
            val.append(val[a] >= val[b])
        elif op == OP_EQ:
            val.append(val[a] == val[b])
        elif op == OP_NE:
            val.append(val[a] != val[b])
        elif op == OP_AND:
            val.append(np.asarray(val[a], dtype=bool) & np.asarray(val[b], dtype=bool))
        elif op == OP_OR:
            val.append(np.asarray(val[a], dtype=bool) | np.asarray(val[b], dtype=bool))
        elif op == OP_NOT:
            val.append(~np.asarray(val[a], dtype=bool))
        else:
            raise ValueError(op)
    ok = np.ones(n, dtype=bool)
    for r in q.roots:
        ok &= np.asarray(val[r], dtype=bool)
    cnt = int(ok.sum())
    if cnt == 0:
        return UNSAT, 0, None
    i = int(np.argmax(ok))
    return SAT, cnt, [int(c[i]) for c in cols]


def int_bruteforce(q, max_bits: int = 22):
    """Every input tuple, in itertools.product order over the declared
    variables (first declared varies slowest).  Returns
    (verdict, number of satisfying tuples, first satisfying tuple or None)."""
    bits = sum(q.var_widths)
    assert bits <= max_bits, f"{bits} input bits is too many for brute force"
    grids = np.meshgrid(*[np.arange(1 << w, dtype=np.int64) for w in q.var_widths],
                        indexing="ij")
    cols = [g.ravel() for g in grids]
    n = cols[0].size if cols else 1
    # exact magnitudes: fall back to Python objects when int64 could overflow
    bound = _magnitude_bounds(q)
    dtype = np.int64 if max(bound + [0]) < (1 << 62) else object
    cols = [c.astype(dtype) for c in cols]
    val = []
    for (op, a, b, w, imm) in q.nodes:
        if op == OP_VAR:
            val.append(cols[imm])
        elif op == OP_CONST:
            val.append(np.full(n, int(imm), dtype=dtype))
        elif op == OP_ADD:
            val.append(val[a] + val[b])
        elif op == OP_SUB:
            val.append(val[a] - val[b])
        elif op == OP_MUL:
            val.append(val[a] * val[b])
        elif op == OP_SHL:
            val.append(val[a] * (1 << int(imm)))
        elif op == OP_UDIV:
            assert (val[a] >= 0).all()
            val.append(val[a] // int(imm))
        elif op == OP_UREM:
            assert (val[a] >= 0).all()
            val.append(val[a] % int(imm))
        elif op == OP_LT:
            val.append(val[a] < val[b])
        elif op == OP_LE:
            val.append(val[a] <= val[b])
        elif op == OP_GT:
            val.append(val[a] > val[b])
        elif op == OP_GE:
            val.append(val[a] >= val[b])
        elif op == OP_EQ:
            val.append(val[a] == val[b])
        elif op == OP_NE:
            val.append(val[a] != val[b])
        elif op == OP_AND:
            val.append(val[a] & val[b])
        elif op == OP_OR:
            val.append(val[a] | val[b])
        elif op == OP_NOT:
            val.append(~val[a])
        else:
            raise ValueError(op)
    ok = np.ones(n, dtype=bool)
    for r in q.roots:
        ok &= np.asarray(val[r], dtype=bool)
    cnt = int(ok.sum())
    if cnt == 0:
        return UNSAT, 0, None
    i = int(np.argmax(ok))
    return SAT, cnt, [int(c[i]) for c in cols]


def _magnitude_bounds(q):
    """Upper bound on |value| of every integer node (booleans: 1)."""
    out = []
    for (op, a, b, w, imm) in q.nodes:
        if op == OP_VAR:
            out.append((1 << q.var_widths[imm]) - 1)
        elif op == OP_CONST:
            out.append(int(imm))
        elif op in (OP_ADD, OP_SUB):
            out.append(out[a] + out[b])
        elif op == OP_MUL:
            out.append(out[a] * out[b])
        elif op == OP_SHL:
            out.append(out[a] << int(imm))
        elif op in (OP_UDIV, OP_UREM):
            out.append(out[a])
        else:
            out.append(1)
    return out


# ------------------------------------------------------------ Tseitin

class _Enc:
    """Plain Tseitin encoder.  Integers are two's complement bit lists,
    least significant bit first, wide enough that no operation overflows."""

    def __init__(self):
        self.n = 0
        self.clauses = []
        self.T = self.new()
        self.clauses.append([self.T])
        self.F = -self.T

    def new(self):
        self.n += 1
        return self.n

    # gates (full equivalence) -----------------------------------------
    def AND(self, a, b):
        if a == self.F or b == self.F or a == -b:
            return self.F
        if a == self.T or a == b:
            return b
        if b == self.T:
            return a
        o = self.new()
        self.clauses += [[-o, a], [-o, b], [o, -a, -b]]
        return o

    def OR(self, a, b):
        return -self.AND(-a, -b)

    def XOR(self, a, b):
        if a == self.F:
            return b
        if b == self.F:
            return a
        if a == self.T:
            return -b
        if b == self.T:
            return -a
        if a == b:
            return self.F
        if a == -b:
            return self.T
        o = self.new()
        self.clauses += [[-o, a, b], [-o, -a, -b], [o, -a, b], [o, a, -b]]
        return o

    def MAJ(self, a, b, c):
        return self.OR(self.OR(self.AND(a, b), self.AND(a, c)), self.AND(b, c))

    # integers ---------------------------------------------------------
    def const(self, v):
        w = max(v.bit_length() + 1, 1) if v >= 0 else (-v - 1).bit_length() + 1
        return [self.T if (v >> i) & 1 else self.F for i in range(w)]

    @staticmethod
    def sext(x, w):
        return x + [x[-1]] * (w - len(x))

    def add(self, x, y):
        w = max(len(x), len(y)) + 1
        x, y = self.sext(x, w), self.sext(y, w)
        out, c = [], self.F
        for i in range(w):
            out.append(self.XOR(self.XOR(x[i], y[i]), c))
            c = self.MAJ(x[i], y[i], c)
        return out

    def add_mod(self, x, y, w):
        out, c = [], self.F
        for i in range(w):
            out.append(self.XOR(self.XOR(x[i], y[i]), c))
            c = self.MAJ(x[i], y[i], c)
        return out

    def neg(self, x):
        w = len(x) + 1
        x = self.sext(x, w)
        inv = [-b for b in x]
        one = [self.T] + [self.F] * (w - 1)
        return self.add_mod(inv, one, w)

    def sub(self, x, y):
        return self.add(x, self.neg(y))

    def mul(self, x, y):
        w = len(x) + len(y)
        x, y = self.sext(x, w), self.sext(y, w)
        acc = [self.F] * w
        for i in range(w):
            pp = [self.F] * i + [self.AND(y[i], x[j]) for j in range(w - i)]
            acc = self.add_mod(acc, pp, w)
        return acc

    def lt(self, x, y):
        return self.sub(x, y)[-1]          # sign bit of x - y

    def eq(self, x, y):
        d = self.sub(x, y)
        r = self.T
        for b in d:
            r = self.AND(r, -b)
        return r


def encode(q):
    """The oracle's own CNF for a query: (CNF, input bit literals per
    declared variable, LSB first)."""
    e = _Enc()
    inputs = []
    for w in q.var_widths:
        inputs.append([e.new() for _ in range(w)])
    val = []
    for (op, a, b, w, imm) in q.nodes:
        if op == OP_VAR:
            val.append(inputs[imm] + [e.F])
        elif op == OP_CONST:
            val.append(e.const(int(imm)))
        elif op == OP_ADD:
            val.append(e.add(val[a], val[b]))
        elif op == OP_SUB:
            val.append(e.sub(val[a], val[b]))
        elif op == OP_MUL:
            val.append(e.mul(val[a], val[b]))
        elif op == OP_SHL:
            val.append([e.F] * int(imm) + val[a])
        elif op in (OP_UDIV, OP_UREM):
            k = int(imm)
            x = val[a]
            # x = qt*k + r with 0 <= r < k; qt and r are functions of x
            qt = [e.new() for _ in range(len(x))] + [e.F]
            r = [e.new() for _ in range(max(k.bit_length(), 1))] + [e.F]
            e.clauses.append([e.eq(x, e.add(e.mul(qt, e.const(k)), r))])
            e.clauses.append([e.lt(r, e.const(k))])
            e.clauses.append([-x[-1]])      # dividend is non-negative
            val.append(qt if op == OP_UDIV else r)
        elif op == OP_LT:
            val.append(e.lt(val[a], val[b]))
        elif op == OP_LE:
            val.append(-e.lt(val[b], val[a]))
        elif op == OP_GT:
            val.append(e.lt(val[b], val[a]))
        elif op == OP_GE:
            val.append(-e.lt(val[a], val[b]))
        elif op == OP_EQ:
            val.append(e.eq(val[a], val[b]))
        elif op == OP_NE:
            val.append(-e.eq(val[a], val[b]))
        elif op == OP_AND:
            val.append(e.AND(val[a], val[b]))
        elif op == OP_OR:
            val.append(e.OR(val[a], val[b]))
        elif op == OP_NOT:
            val.append(-val[a])
        else:
            raise ValueError(op)
    for r in q.roots:
        e.clauses.append([val[r]])
    # drop clauses made trivial by constants; keep every variable
    clauses = []
    for cl in e.clauses:
        if any(l == e.T for l in cl):
            if cl == [e.T]:
                clauses.append(cl)
            continue
        cl = [l for l in cl if l != e.F]
        seen, out, taut = set(), [], False
        for l in cl:
            if -l in seen:
                taut = True
            if l not in seen:
                seen.add(l)
                out.append(l)
        if not taut:
            clauses.append(out)
    return CNF.from_clauses(e.n, clauses, q.name), inputs


def decode_inputs(model, inputs):
    return [sum(1 << i for i, l in enumerate(bits) if model[l] == 1)
            for bits in inputs]


# ------------------------------------------------------------ root check

def _poly_of(q):
    """Polynomial normal form of every integer node: dict monomial -> coef,
    a monomial being a sorted tuple of atom keys (() is the constant).
    Atoms are inputs ('v', i) or opaque non-polynomial nodes ('n', node)."""
    polys = []

    def padd(p, r, s=1):
        out = dict(p)
        for m, c in r.items():
            out[m] = out.get(m, 0) + s * c
            if out[m] == 0:
                del out[m]
        return out

    def pmul(p, r):
        out = {}
        for m1, c1 in p.items():
            for m2, c2 in r.items():
                m = tuple(sorted(m1 + m2))
                out[m] = out.get(m, 0) + c1 * c2
                if out[m] == 0:
                    del out[m]
        return out

    for i, (op, a, b, w, imm) in enumerate(q.nodes):
        if op == OP_VAR:
            polys.append({(("v", int(imm)),): 1})
        elif op == OP_CONST:
            polys.append({(): int(imm)} if imm else {})
        elif op == OP_ADD:
            polys.append(padd(polys[a], polys[b]))
        elif op == OP_SUB:
            polys.append(padd(polys[a], polys[b], -1))
        elif op == OP_MUL:
            polys.append(pmul(polys[a], polys[b]))
        elif op == OP_SHL:
            polys.append({m: c << int(imm) for m, c in polys[a].items()})
        elif op in (OP_UDIV, OP_UREM):
            polys.append({(("n", i),): 1})
        else:
            polys.append(None)
    return polys


def _atom_range(q, key, polys):
    """Interval of an atom from the input domains (inputs) or of an opaque
    node (quotient / remainder of a non-negative value)."""
    kind, i = key
    if kind == "v":
        return 0, (1 << q.var_widths[i]) - 1
    op, a, _, _, imm = q.nodes[i]
    lo, hi = _poly_range(q, polys[a], polys)
    lo = max(lo, 0)
    if op == OP_UDIV:
        return lo // imm, hi // imm
    return 0, min(imm - 1, hi)


def _poly_range(q, p, polys):
    lo = hi = 0
    for m, c in p.items():
        mlo, mhi = 1, 1
        for key in m:
            alo, ahi = _atom_range(q, key, polys)
            cands = [mlo * alo, mlo * ahi, mhi * alo, mhi * ahi]
            mlo, mhi = min(cands), max(cands)
        if c >= 0:
            lo, hi = lo + c * mlo, hi + c * mhi
        else:
            lo, hi = lo + c * mhi, hi + c * mlo
    return lo, hi


def _substitute(p, atom, expr):
    """p with every occurrence of atom replaced by the polynomial expr."""
    out = {}
    for m, c in p.items():
        k = m.count(atom)
        term = {tuple(x for x in m if x != atom): c}
        for _ in range(k):
            nxt = {}
            for m1, c1 in term.items():
                for m2, c2 in expr.items():
                    mm = tuple(sorted(m1 + m2))
                    nxt[mm] = nxt.get(mm, 0) + c1 * c2
            term = nxt
        for mm, cc in term.items():
            out[mm] = out.get(mm, 0) + cc
    return {m: c for m, c in out.items() if c != 0}


def _substitute_all(p, subs):
    for atom, expr in subs:
        p = _substitute(p, atom, expr)
    return p


# Linear relaxation.  A constraint is (coefs, const) meaning
# sum(coefs[m] * m) + const >= 0 over monomials m, coefs coprime integers,
# const a Fraction.  Rational feasibility is what Fourier-Motzkin decides;
# every derived constraint is a non-negative combination of the inputs.
FM_CAP = 20000


def _fm_norm(coefs, const):
    coefs = {m: c for m, c in coefs.items() if c != 0}
    g = 0
    for c in coefs.values():
        g = gcd(g, abs(c))
    if g > 1:
        coefs = {m: c // g for m, c in coefs.items()}
        const = Fraction(const) / g
    return coefs, Fraction(const)


def fm_infeasible(constraints):
    """True iff the system {sum c_m m + c0 >= 0} has no rational solution.
    None when the elimination exceeds FM_CAP constraints (undecided)."""
    best = {}

    def add(pool, coefs, const):
        coefs, const = _fm_norm(coefs, const)
        if not coefs:
            return const < 0            # a contradiction
        key = tuple(sorted(coefs.items()))
        if key not in pool or const < pool[key]:
            pool[key] = const
        return False

    for coefs, const in constraints:
        if add(best, coefs, const):
            return True
    pool = best
    while pool:
        if len(pool) > FM_CAP:
            return None
        vars_ = sorted({m for key in pool for m, _ in key})
        if not vars_:
            return False

        def cost(x):
            pos = sum(1 for key in pool if dict(key).get(x, 0) > 0)
            neg = sum(1 for key in pool if dict(key).get(x, 0) < 0)
            return pos * neg - pos - neg
        x = min(vars_, key=lambda v: (cost(v), v))
        pos, neg, nxt = [], [], {}
        for key, const in pool.items():
            c = dict(key).get(x, 0)
            if c > 0:
                pos.append((dict(key), const))
            elif c < 0:
                neg.append((dict(key), const))
            else:
                nxt[key] = const
        for pc, pk in pos:
            a = pc[x]
            for nc, nk in neg:
                b = -nc[x]
                comb = {}
                for m, c in pc.items():
                    comb[m] = comb.get(m, 0) + b * c
                for m, c in nc.items():
                    comb[m] = comb.get(m, 0) + a * c
                comb.pop(x, None)
                if add(nxt, comb, b * pk + a * nk):
                    return True
        pool = nxt
    return False


def _lp_check(q, polys, facts):
    """Facts (poly, 'ge'|'eq') -> True if their linear relaxation with atom
    products and monomial ranges is infeasible over the rationals."""
    present = {m for p, _ in facts for m in p if m != ()}
    atoms = sorted({a for m in present for a in m})
    rows = []
    for p, kind in facts:
        prods = [p]
        for z in atoms:
            zp = {tuple(sorted(m + (z,))): c for m, c in p.items()}
            if all(m in present for m in zp):
                prods.append(zp)
        for r in prods:
            coefs = {m: c for m, c in r.items() if m != ()}
            const = r.get((), 0)
            rows.append((coefs, const))
            if kind == "eq":
                rows.append(({m: -c for m, c in coefs.items()}, -const))
    for m in present:
        lo, hi = _poly_range(q, {m: 1}, polys)
        rows.append(({m: 1}, -lo))
        rows.append(({m: -1}, hi))
    return fm_infeasible(rows) is True


def root_check(q):
    """UNSAT if the root conjunction bounds one polynomial by an empty
    interval; else None (undecided)."""
    polys = _poly_of(q)
    facts = []          # (poly, kind) meaning poly >= 0 ('ge') or == 0 ('eq')

    def diff(a, b, k=0):
        p = dict(polys[a])
        for m, c in polys[b].items():
            p[m] = p.get(m, 0) - c
            if p[m] == 0:
                del p[m]
        if k:
            p[()] = p.get((), 0) + k
            if p[()] == 0:
                del p[()]
        return p

    def collect(i, positive):
        op, a, b, _, _ = q.nodes[i]
        if op == OP_AND and positive:
            collect(a, True)
            collect(b, True)
        elif op == OP_OR and not positive:
            collect(a, False)
            collect(b, False)
        elif op == OP_NOT:
            collect(a, not positive)
        elif op in (OP_LT, OP_LE, OP_GT, OP_GE):
            # a < b  <=>  b - a - 1 >= 0 ; negation flips to a >= b
            if op == OP_LT:
                p = diff(b, a, -1) if positive else diff(a, b)
            elif op == OP_LE:
                p = diff(b, a) if positive else diff(a, b, -1)
            elif op == OP_GT:
                p = diff(a, b, -1) if positive else diff(b, a)
            else:
                p = diff(a, b) if positive else diff(b, a, -1)
            facts.append((p, "ge"))
        elif op == OP_EQ and positive:
            facts.append((diff(a, b), "eq"))
        elif op == OP_NE and not positive:
            facts.append((diff(a, b), "eq"))

    for r in q.roots:
        collect(r, True)

    # Root equalities that define an atom linearly (coefficient +-1, the
    # atom in no other monomial) are used to eliminate it from every fact;
    # the rewritten facts are implied by the originals and join them.
    subs = []                       # (atom, polynomial free of pivots)
    for p, kind in facts:
        if kind != "eq":
            continue
        p = _substitute_all(p, subs)
        pivot = None
        for m, c in p.items():
            if len(m) == 1 and abs(c) == 1 and \
                    all(m[0] not in m2 for m2 in p if m2 != m):
                pivot = (m[0], c)
                break
        if pivot is None:
            continue
        atom, c = pivot
        # atom = -(p - c*atom) / c
        expr = {m: -cc * c for m, cc in p.items() if m != (atom,)}
        subs = [(a, _substitute(e, atom, expr)) for a, e in subs]
        subs.append((atom, expr))
    facts = facts + [(_substitute_all(p, subs), kind) for p, kind in facts]

    bounds = {}   # normalised polynomial -> [lo, hi] (None = unbounded)
    for p, kind in facts:
        c0 = p.get((), 0)
        rest = {m: c for m, c in p.items() if m != ()}
        if not rest:
            if (kind == "ge" and c0 < 0) or (kind == "eq" and c0 != 0):
                return UNSAT
            continue
        g = 0
        for c in rest.values():
            g = gcd(g, abs(c))
        lead = min(rest)                      # canonical leading monomial
        s = 1 if rest[lead] > 0 else -1
        key = tuple(sorted((m, c * s // g) for m, c in rest.items()))
        # rest = s*g*key ;  constraint: s*g*key + c0 >= 0  (or == 0)
        lo, hi = None, None
        if kind == "eq":
            if c0 % g:
                return UNSAT
            v = -c0 // g * s
            lo = hi = v
        elif s > 0:
            lo = -((c0) // g)                 # key >= ceil(-c0/g)
        else:
            hi = c0 // g                      # key <= floor(c0/g)
        cur = bounds.setdefault(key, [None, None])
        if lo is not None:
            cur[0] = lo if cur[0] is None else max(cur[0], lo)
        if hi is not None:
            cur[1] = hi if cur[1] is None else min(cur[1], hi)
    for key, (lo, hi) in bounds.items():
        rlo, rhi = _poly_range(q, dict(key), polys)
        lo = rlo if lo is None else max(lo, rlo)
        hi = rhi if hi is None else min(hi, rhi)
        if lo > hi:
            return UNSAT
    if _lp_check(q, polys, facts):
        return UNSAT
    return None


# ------------------------------------------------------------ decide

def decide(q, max_nodes: int = cnf_ref.DEFAULT_NODES, candidate=None):
    """(verdict, witness input values or None, how) for one query.

    Root check, else DPLL on the oracle's own encoding.  When DPLL runs out
    of its node budget and a candidate input tuple is given, the candidate
    decides by the definition itself: SAT iff it satisfies every root under
    exact integer arithmetic ("checked"); otherwise the verdict is UNKNOWN."""
    if root_check(q) == UNSAT:
        return UNSAT, None, "root"
    cnf, inputs = encode(q)
    verdict, model, _ = cnf_ref.solve(cnf, max_nodes)
    if verdict == SAT:
        return SAT, decode_inputs(model, inputs), "dpll"
    if verdict == UNKNOWN and candidate is not None and int_eval(q, candidate):
        return SAT, list(candidate), "checked"
    return verdict, None, "dpll"


def product_order_inputs(q):
    """All input tuples in brute-force order (tiny queries only)."""
    return itertools.product(*[range(1 << w) for w in q.var_widths])
