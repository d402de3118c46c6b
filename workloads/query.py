"""Query DAG format and a small builder for it.

A query is the constraint set that the bounds analysis emits for one static
memory access (its constraint kinds 1-3, Sec. 4.1 and Sec. 5.2): thread and
block ids below their dimensions, equalities that define offset, size, grid
dimensions and asserts through expression trees, and the out-of-bounds test
``offset >= size``.  Expression trees (Sec. 5.1, Fig. 8) become one DAG per
query: leaves are constants or unknown inputs, inner nodes are operators, and
an input that appears in several trees is one node (the paper identifies
variables across trees by their IR value).

This module only *describes* queries.  It evaluates nothing: the exact
integer meaning lives in the oracle, the bit-level meaning in the library.

Node record (24 bytes, little endian, same layout as ``scuba_node`` in
``include/scuba.h``)::

    op:u32  a:u32  b:u32  width:u32  imm:u64

* ``a`` and ``b`` index earlier nodes of the same query (topological order).
* ``VAR``: an unknown input, unsigned, ``0 <= x < 2**width`` with
  ``1 <= width <= 64``; ``imm`` is its declaration number (0, 1, ...).
* ``CONST``: the unsigned integer ``imm``.
* ``SHL`` / ``UDIV`` / ``UREM``: operand ``a`` with the constant ``imm``
  (shift amount, or a divisor > 0).  ``UDIV``/``UREM`` need ``a >= 0``.
* comparisons and boolean connectives produce booleans; ``roots`` lists the
  boolean nodes that must all hold.

Arithmetic is over the unbounded integers (no wrap-around); a ``SUB`` may go
negative.
"""
from __future__ import annotations

import numpy as np

OP_VAR, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_SHL, OP_UDIV, OP_UREM = range(8)
OP_LT, OP_LE, OP_GT, OP_GE, OP_EQ, OP_NE = range(8, 14)
OP_AND, OP_OR, OP_NOT = range(14, 17)

OP_NAMES = {
    OP_VAR: "var", OP_CONST: "const", OP_ADD: "add", OP_SUB: "sub",
    OP_MUL: "mul", OP_SHL: "shl", OP_UDIV: "udiv", OP_UREM: "urem",
    OP_LT: "lt", OP_LE: "le", OP_GT: "gt", OP_GE: "ge", OP_EQ: "eq",
    OP_NE: "ne", OP_AND: "and", OP_OR: "or", OP_NOT: "not",
}
INT_OPS = (OP_VAR, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_SHL, OP_UDIV, OP_UREM)
CMP_OPS = (OP_LT, OP_LE, OP_GT, OP_GE, OP_EQ, OP_NE)
BOOL_OPS = CMP_OPS + (OP_AND, OP_OR, OP_NOT)

NODE_DTYPE = np.dtype([("op", "<u4"), ("a", "<u4"), ("b", "<u4"),
                       ("width", "<u4"), ("imm", "<u8")])
assert NODE_DTYPE.itemsize == 24


class Expr:
    """Handle to one node of a :class:`Query`; operators append nodes."""

    __slots__ = ("q", "i")

    def __init__(self, q: "Query", i: int):
        self.q, self.i = q, i

    # integer operators -------------------------------------------------
    def _lift(self, o):
        if isinstance(o, Expr):
            assert o.q is self.q, "nodes of different queries"
            return o
        if isinstance(o, (int, np.integer)) and not isinstance(o, bool):
            return self.q.const(int(o))
        raise TypeError(f"cannot use {type(o)} in a query")

    def __add__(self, o): return self.q._node(OP_ADD, self, self._lift(o))
    def __radd__(self, o): return self.q._node(OP_ADD, self._lift(o), self)
    def __sub__(self, o): return self.q._node(OP_SUB, self, self._lift(o))
    def __rsub__(self, o): return self.q._node(OP_SUB, self._lift(o), self)
    def __mul__(self, o): return self.q._node(OP_MUL, self, self._lift(o))
    def __rmul__(self, o): return self.q._node(OP_MUL, self._lift(o), self)

    def __lshift__(self, k: int): return self.q._node(OP_SHL, self, imm=int(k))

    def __floordiv__(self, k: int):
        assert int(k) > 0
        return self.q._node(OP_UDIV, self, imm=int(k))

    def __mod__(self, k: int):
        assert int(k) > 0
        return self.q._node(OP_UREM, self, imm=int(k))

    # comparisons -------------------------------------------------------
    def __lt__(self, o): return self.q._node(OP_LT, self, self._lift(o))
    def __le__(self, o): return self.q._node(OP_LE, self, self._lift(o))
    def __gt__(self, o): return self.q._node(OP_GT, self, self._lift(o))
    def __ge__(self, o): return self.q._node(OP_GE, self, self._lift(o))
    def eq(self, o): return self.q._node(OP_EQ, self, self._lift(o))
    def ne(self, o): return self.q._node(OP_NE, self, self._lift(o))

    # boolean connectives ----------------------------------------------
    def __and__(self, o): return self.q._node(OP_AND, self, o)
    def __or__(self, o): return self.q._node(OP_OR, self, o)
    def __invert__(self): return self.q._node(OP_NOT, self)

    def __bool__(self):
        raise TypeError("query expressions have no Python truth value")

    __hash__ = object.__hash__


class Query:
    """A DAG of nodes plus the list of boolean roots asserted true."""

    def __init__(self, name: str = ""):
        self.name = name
        self.nodes: list[tuple[int, int, int, int, int]] = []
        self.roots: list[int] = []
        self.var_names: list[str] = []
        self.var_widths: list[int] = []
        self._consts: dict[int, int] = {}

    def _node(self, op, a=None, b=None, width=0, imm=0) -> Expr:
        ia = a.i if a is not None else 0
        ib = b.i if b is not None else 0
        self.nodes.append((op, ia, ib, width, imm))
        return Expr(self, len(self.nodes) - 1)

    def var(self, name: str, width: int) -> Expr:
        assert 1 <= width <= 64, "input widths are 1..64 bits"
        assert name not in self.var_names, f"duplicate variable {name}"
        e = self._node(OP_VAR, width=width, imm=len(self.var_names))
        self.var_names.append(name)
        self.var_widths.append(width)
        return e

    def const(self, value: int) -> Expr:
        assert 0 <= value < 2 ** 64, "constants are unsigned 64-bit"
        if value not in self._consts:
            self._consts[value] = self._node(OP_CONST, imm=value).i
        return Expr(self, self._consts[value])

    def require(self, cond: Expr) -> None:
        """Assert a boolean node (a guard, an assert, a bound, the OOB test)."""
        assert cond.q is self
        self.roots.append(cond.i)

    def arrays(self):
        """(nodes: NODE_DTYPE array, roots: uint32 array, var_names)."""
        nodes = np.array(self.nodes, dtype=NODE_DTYPE) if self.nodes else \
            np.zeros(0, dtype=NODE_DTYPE)
        return nodes, np.array(self.roots, dtype=np.uint32), list(self.var_names)

    @property
    def n_vars(self) -> int:
        return len(self.var_names)

    @property
    def input_bits(self) -> int:
        return sum(self.var_widths)

    def __repr__(self):
        return (f"Query({self.name!r}, nodes={len(self.nodes)}, "
                f"roots={len(self.roots)}, vars={self.var_names})")
