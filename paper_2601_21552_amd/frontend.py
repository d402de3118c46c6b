"""Query front-end: host and kernel analysis of a program into one OOB query
per memory instruction and launch (paper Sec. 5.1, Fig. 8 and Fig. 9a/9b;
constraints as in Sec. 5.2).

Host pass (Fig. 9a): the size of every ``malloc`` as an expression tree
over the inputs; for every launch the grid and block dimensions, the
arguments (a pointer argument stands for its allocation's size tree, a scalar
for its own tree) and the dynamic shared size; the asserts met so far.

Kernel pass (Fig. 9b): static arrays with their size trees; the dynamic
shared base and its partitions in program order, the size of each part
being the next part's offset minus its own and the last part's the dynamic
shared size minus its offset; every load, store and atomic with its data
structure, its offset tree and the guards and loop bounds that dominate it.

One query per (launch, memory instruction):
* kind 1: ``threadIdx.a < blockDim.a`` and ``blockIdx.a < gridDim.a`` on
  every axis whose dimension is not the literal 1;
* kind 3: offset, size and grid dimensions are their trees, shared in one
  DAG so that a program variable is one node wherever it is used (the
  paper's IR-value identity), plus the asserts that precede the launch and
  the conditions of the host branches that hold it;
* the guards and loop bounds on the access's path;
* kind 2: ``offset >= size`` (upper), or ``offset < 0`` (lower bound).

Reading: an assert after a launch cannot stop that launch, so only the
asserts before it join its queries.  Ids and loop counters are unsigned
inputs as wide as the largest value their bound can take (an interval
bound over the trees).  Programs whose ``/`` or ``%`` may see a negative
left operand are rejected: unsigned division of a negative value has no
meaning in the query format.
"""
from __future__ import annotations

from dataclasses import dataclass

from workloads.program import AXES, Program, expr_text
from workloads.query import Query


class FrontendError(ValueError):
    pass


@dataclass
class AccessQuery:
    key: tuple          # (launch index, kernel, access index, "upper" | "lower")
    query: Query
    region: str         # "global", "static" or "partition"
    access: str         # the access, printed

    @property
    def name(self):
        return self.query.name


def _lit1(e):
    return e == ("num", 1)


class _Launch:
    """Symbolic context of one launch: expression trees built into one query."""

    def __init__(self, prog: Program, launch, q: Query):
        self.p, self.q = prog, q
        _, self.kname, self.grid, self.block, shm, args = launch
        self.shm = shm if shm is not None else ("num", 0)
        params, self.body = prog.kernels[self.kname]
        self.host_defs = {}
        for s in prog.host:
            if s[0] in ("input", "let", "malloc"):
                self.host_defs[s[1]] = s
        self.ptr = {}       # kernel parameter -> malloc size tree (host scope)
        self.scalar = {}    # kernel parameter -> argument tree (host scope)
        for name, a in zip(params, args):
            d = self.host_defs.get(a[1]) if a[0] == "ref" else None
            if d is not None and d[0] == "malloc":
                self.ptr[name] = d[2]
            else:
                self.scalar[name] = a
        self.klets = {}     # kernel let name -> tree (kernel scope)
        self.loops = {}     # loop counter -> bound tree (kernel scope)
        self.statics, self.parts = {}, []   # name -> size tree; [(name, offset tree)]
        self._sym, self._rng = {}, {}

    # ---- name resolution ---------------------------------------------
    def _lookup(self, name, scope):
        """('tree', expr, scope) or ('input' | 'id' | 'loop', ...)."""
        if scope == "kernel":
            if name in self.klets:
                return ("tree", self.klets[name], "kernel")
            if name in self.loops:
                return ("loop", name)
            if name in self.scalar:
                return ("tree", self.scalar[name], "host")
            if name in self.ptr:
                raise FrontendError(f"{self.p.name}: pointer {name} used as a value")
            if "." in name:
                b, a = name.split(".")
                ax = AXES.index(a)
                if b == "blockDim":
                    return ("tree", self.block[ax], "host")
                if b == "gridDim":
                    return ("tree", self.grid[ax], "host")
                return ("id", b, ax)
        d = self.host_defs[name]
        if d[0] == "input":
            return ("input", name, d[2])
        if d[0] == "malloc":
            raise FrontendError(f"{self.p.name}: pointer {name} used as a value")
        return ("tree", d[2], "host")

    # ---- interval bounds (for widths and the division check) --------
    def rng(self, e, scope):
        key = (e, scope)
        if key in self._rng:
            return self._rng[key]
        t = e[0]
        if t == "num":
            r = (e[1], e[1])
        elif t == "ref":
            d = self._lookup(e[1], scope)
            if d[0] == "tree":
                r = self.rng(d[1], d[2])
            elif d[0] == "input":
                r = (0, 2 ** d[2] - 1)
            elif d[0] == "loop":
                r = (0, max(self.rng(self.loops[d[1]], "kernel")[1] - 1, 0))
            else:
                dim = (self.block if d[1] == "threadIdx" else self.grid)[d[2]]
                r = (0, max(self.rng(dim, "host")[1] - 1, 0))
        elif t == "not":
            r = (0, 1)
        else:
            op, (alo, ahi) = e[1], self.rng(e[2], scope)
            if op in ("/", "%", "<<"):
                k = e[3][1]
                if op != "<<" and alo < 0:
                    raise FrontendError(f"{self.p.name}: {expr_text(e)} may divide a negative value")
                if op == "/":
                    r = (alo // k, ahi // k)
                elif op == "%":
                    r = (alo, ahi) if ahi < k else (0, k - 1)
                else:
                    r = (alo << k, ahi << k)
            else:
                blo, bhi = self.rng(e[3], scope)
                if op == "+":
                    r = (alo + blo, ahi + bhi)
                elif op == "-":
                    r = (alo - bhi, ahi - blo)
                elif op == "*":
                    c = (alo * blo, alo * bhi, ahi * blo, ahi * bhi)
                    r = (min(c), max(c))
                else:
                    r = (0, 1)
        self._rng[key] = r
        return r

    def _width(self, hi):
        w = max(1, (max(hi, 1) - 1).bit_length())
        if w > 64:
            raise FrontendError(f"{self.p.name}: an id or loop counter may exceed 64 bits")
        return w

    # ---- expression trees into the query ----------------------------
    def id_var(self, b, ax):
        dim = (self.block if b == "threadIdx" else self.grid)[ax]
        if _lit1(dim):
            return self.q.const(0)
        name = f"{b}.{AXES[ax]}"
        if name not in self._sym:
            self._sym[name] = self.q.var(name, self._width(self.rng(dim, "host")[1]))
        return self._sym[name]

    def sym(self, e, scope):
        key = (e, scope)
        if key in self._sym:
            return self._sym[key]
        q, t = self.q, e[0]
        if t == "num":
            v = q.const(e[1])
        elif t == "ref":
            d = self._lookup(e[1], scope)
            if d[0] == "tree":
                v = self.sym(d[1], d[2])
            elif d[0] == "input":
                if ("in", d[1]) not in self._sym:
                    self._sym[("in", d[1])] = q.var(d[1], d[2])
                v = self._sym[("in", d[1])]
            elif d[0] == "loop":
                v = self._sym[("loop", d[1])]
            else:
                v = self.id_var(d[1], d[2])
        elif t == "not":
            v = ~self.sym(e[1], scope)
        else:
            op = e[1]
            a = self.sym(e[2], scope)
            if op in ("/", "%", "<<"):
                self.rng(e, scope)   # rejects a possibly negative dividend
                k = e[3][1]
                v = a // k if op == "/" else a % k if op == "%" else a << k
            else:
                b = self.sym(e[3], scope)
                v = {"+": lambda: a + b, "-": lambda: a - b, "*": lambda: a * b,
                     "<": lambda: a < b, "<=": lambda: a <= b, ">": lambda: a > b,
                     ">=": lambda: a >= b, "==": lambda: a.eq(b), "!=": lambda: a.ne(b),
                     "&&": lambda: a & b, "||": lambda: a | b}[op]()
        self._sym[key] = v
        return v

    def loop_var(self, name, bound):
        self.loops[name] = bound
        hi = self.rng(bound, "kernel")[1]
        self._sym[("loop", name)] = self.q.var(f"for:{name}", self._width(hi))
        return self._sym[("loop", name)]


def _kernel_accesses(body):
    """Every access of a kernel body with its path: a list of
    ('if', cond, taken) / ('loop', name, bound) steps, plus the declarations
    met before it: (access stmt, path, lets, statics, dyn base, parts)."""
    out = []
    lets, statics, parts = {}, {}, []

    def walk(stmts, path):
        path = list(path)
        for s in stmts:
            k = s[0]
            if k == "let":
                lets[s[1]] = s[2]
            elif k == "static":
                statics[s[1]] = s[2]
            elif k == "dynshared":
                parts.append((s[1], ("num", 0)))
            elif k == "partition":
                parts.append((s[1], s[3]))
            elif k == "access":
                out.append((s, tuple(path)))
            elif k == "if":
                walk(s[2], path + [("if", s[1], True)])
                walk(s[3], path + [("if", s[1], False)])
            elif k == "guard":
                path.append(("if", s[1], True))
            elif k == "for":
                walk(s[3], path + [("loop", s[1], s[2])])
    walk(body, [])
    return out, lets, statics, parts


def _host_launches(stmts, asserts, conds, out):
    """(launch, asserts before it, host branch conditions on its path) in
    program order, then-branches first."""
    for s in stmts:
        if s[0] == "assert":
            asserts.append(s[1])
        elif s[0] == "launch":
            out.append((s, list(asserts), list(conds)))
        elif s[0] == "hif":
            _host_launches(s[2], asserts, conds + [(s[1], True)], out)
            _host_launches(s[3], asserts, conds + [(s[1], False)], out)
    return out


def analyse(prog: Program, lower: bool = False) -> list[AccessQuery]:
    """One query per (launch, memory instruction), in launch then program
    order; with ``lower`` each access also gets its lower-bound query."""
    out = []
    for li, (s, asserts, conds) in enumerate(_host_launches(prog.host, [], [], [])):
        accesses, lets, statics, parts = _kernel_accesses(prog.kernels[s[1]][1])
        for ai, (acc, path) in enumerate(accesses):
            for bound in (("upper", "lower") if lower else ("upper",)):
                key = (li, s[1], ai, bound)
                q = Query(f"{prog.name}:L{li}:{s[1]}:{ai}:{bound}")
                L = _Launch(prog, s, q)
                L.klets = dict(lets)
                # kind 1 on every axis whose dimension is not the literal 1
                for ax in range(3):
                    for b, dims in (("threadIdx", L.block), ("blockIdx", L.grid)):
                        if not _lit1(dims[ax]):
                            q.require(L.id_var(b, ax) < L.sym(dims[ax], "host"))
                for a in asserts:
                    q.require(L.sym(a, "host"))
                for c, taken in conds:
                    hc = L.sym(c, "host")
                    q.require(hc if taken else ~hc)
                for step in path:
                    if step[0] == "if":
                        c = L.sym(step[1], "kernel")
                        q.require(c if step[2] else ~c)
                    else:
                        v = L.loop_var(step[1], step[2])
                        q.require(v < L.sym(step[2], "kernel"))
                _, op, ds, idx = acc
                offset = L.sym(idx, "kernel")
                if ds in L.ptr:
                    region, size = "global", L.sym(L.ptr[ds], "host")
                elif ds in statics:
                    region, size = "static", L.sym(statics[ds], "kernel")
                else:
                    names = [p[0] for p in parts]
                    if ds not in names:
                        raise FrontendError(f"{prog.name}: {ds} is not a buffer")
                    j = names.index(ds)
                    nxt = parts[j + 1][1] if j + 1 < len(parts) else L.shm
                    scope_n = "kernel" if j + 1 < len(parts) else "host"
                    region = "partition"
                    size = L.sym(nxt, scope_n) - L.sym(parts[j][1], "kernel")
                q.require(offset >= size if bound == "upper" else offset < 0)
                out.append(AccessQuery(key, q, region, f"{op} {ds}[{expr_text(idx)}]"))
    return out
