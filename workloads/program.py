"""Small GPU programs in a C-like language, for the query front-end.

A program is what the bounds analysis reads (Sec. 5.1): host code that takes
unknown user inputs, allocates global buffers, asserts conditions and
launches kernels, and kernel code that allocates static shared or local
arrays, carves the dynamic shared buffer into partitions and accesses memory
at computed offsets.  This module holds only the syntax: a tokenizer, a
parser into plain tuples, a printer and seeded program generators.  It
evaluates nothing; the symbolic meaning is in the library's front-end and the
concrete one in the oracle's interpreter.

Grammar (statements are keyword-led; newlines are plain white space; ``//``
starts a comment)::

    program  := { host | kernel }
    host     := 'input' NAME ':' INT               unknown unsigned input of INT bits
              | 'let' NAME '=' expr
              | 'malloc' NAME '=' expr              global buffer of expr elements
              | 'assert' expr
              | 'free' NAME                          release a global buffer
              | launch
              | 'if' '(' expr ')' hblock ['else' hblock]
    launch   := 'launch' NAME 'grid' dims 'block' dims ['shm' '(' expr ')']
                       'args' '(' [expr {',' expr}] ')'
    hblock   := '{' { 'free' NAME | launch | 'if' ... } '}'   (no inputs, lets,
                                                    mallocs or asserts in branches)
    dims     := '(' expr [',' expr [',' expr]] ')'   missing axes are 1
    kernel   := 'kernel' NAME '(' [NAME {',' NAME}] ')' block
    block    := '{' { kstmt } '}'
    kstmt    := 'let' NAME '=' expr
              | ('shared' | 'local') NAME '[' expr ']'    static array (constant size)
              | 'dynshared' NAME                           base of the dynamic shared buffer
              | 'partition' NAME '=' NAME '+' expr         a part starting at that offset
              | ('load' | 'store' | 'atomic') NAME '[' expr ']'
              | 'free' NAME                                release a pointer parameter
              | 'if' '(' expr ')' block ['else' block]
              | 'guard' expr        the rest of the block runs only where expr holds
              | 'for' NAME '<' expr block                  NAME = 0, 1, ..., expr - 1

Expressions use C's operators and precedence (``|| && == != < <= > >= <<
+ - * / % !``), integer literals, names, and ``threadIdx``, ``blockIdx``,
``blockDim``, ``gridDim`` with ``.x``/``.y``/``.z``.  Arithmetic is over the
unbounded integers; ``/``, ``%`` and ``<<`` take a constant right operand.
All sizes and offsets count elements.  Launches are numbered in program
order, the then-branch of a host ``if`` before its else-branch.

Parsed form: expressions are tuples ``("num", v)``, ``("ref", name)`` (a
builtin is the name ``"threadIdx.x"`` etc.), ``("bin", op, a, b)``,
``("not", a)``; statements are tuples led by their keyword (see ``parse``).
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field

import numpy as np

BUILTINS = tuple(f"{b}.{a}" for b in ("threadIdx", "blockIdx", "blockDim", "gridDim")
                 for a in "xyz")
AXES = "xyz"

_TOKEN = re.compile(r"\s*(?:(//[^\n]*)|(\d+)|([A-Za-z_][A-Za-z_0-9]*(?:\.[A-Za-z]+)?)|"
                    r"(\|\||&&|==|!=|<=|>=|<<|[-+*/%<>!=(){}\[\],:]))")
_KEYWORDS = {"input", "let", "malloc", "assert", "launch", "grid", "block", "shm", "args",
             "kernel", "shared", "local", "dynshared", "partition", "load", "store",
             "atomic", "if", "else", "guard", "for", "free"}
# C precedence, loosest first
_LEVELS = [("||",), ("&&",), ("==", "!="), ("<", "<=", ">", ">="), ("<<",), ("+", "-"),
           ("*", "/", "%")]


class ParseError(ValueError):
    pass


def tokenize(text: str):
    out, pos = [], 0
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise ParseError(f"bad character at {text[pos:pos + 20]!r}")
        pos = m.end()
        if m.group(1):
            continue
        if m.group(2):
            out.append(("int", int(m.group(2))))
        elif m.group(3):
            w = m.group(3)
            if "." in w and w not in BUILTINS:
                raise ParseError(f"unknown builtin {w}")
            out.append(("kw" if w in _KEYWORDS else "name", w))
        else:
            out.append(("op", m.group(4)))
    return out


class _Parser:
    def __init__(self, text):
        self.t = tokenize(text)
        self.i = 0

    def peek(self, k=0):
        return self.t[self.i + k] if self.i + k < len(self.t) else ("eof", None)

    def take(self, kind=None, val=None):
        tok = self.peek()
        if (kind and tok[0] != kind) or (val is not None and tok[1] != val):
            raise ParseError(f"expected {val or kind}, got {tok[1]!r} (token {self.i})")
        self.i += 1
        return tok[1]

    def accept(self, val):
        if self.peek()[1] == val and self.peek()[0] in ("op", "kw"):
            self.i += 1
            return True
        return False

    # expressions -------------------------------------------------------
    def expr(self, level=0):
        if level == len(_LEVELS):
            return self.unary()
        a = self.expr(level + 1)
        while self.peek()[0] == "op" and self.peek()[1] in _LEVELS[level]:
            op = self.take()
            b = self.expr(level + 1)
            a = ("bin", op, a, b)
        return a

    def unary(self):
        tok = self.peek()
        if tok == ("op", "!"):
            self.take()
            return ("not", self.unary())
        if tok == ("op", "("):
            self.take()
            e = self.expr()
            self.take("op", ")")
            return e
        if tok[0] == "int":
            self.take()
            return ("num", tok[1])
        if tok[0] == "name":
            self.take()
            return ("ref", tok[1])
        raise ParseError(f"expected an expression, got {tok[1]!r}")

    def dims(self):
        self.take("op", "(")
        d = [self.expr()]
        while self.accept(","):
            d.append(self.expr())
        self.take("op", ")")
        if len(d) > 3:
            raise ParseError("at most three axes")
        return tuple(d) + (("num", 1),) * (3 - len(d))

    # statements --------------------------------------------------------
    def host(self):
        kw = self.take("kw")
        if kw == "input":
            name = self.take("name")
            self.take("op", ":")
            return ("input", name, self.take("int"))
        if kw in ("let", "malloc"):
            name = self.take("name")
            self.take("op", "=")
            return (kw, name, self.expr())
        if kw == "assert":
            return ("assert", self.expr())
        if kw == "free":
            return ("free", self.take("name"))
        if kw == "if":
            self.take("op", "(")
            c = self.expr()
            self.take("op", ")")
            then = self.hblock()
            other = self.hblock() if self.accept("else") else ()
            return ("hif", c, then, other)
        if kw == "launch":
            kname = self.take("name")
            self.take("kw", "grid")
            grid = self.dims()
            self.take("kw", "block")
            block = self.dims()
            shm = None
            if self.accept("shm"):
                self.take("op", "(")
                shm = self.expr()
                self.take("op", ")")
            self.take("kw", "args")
            self.take("op", "(")
            args = []
            if not self.accept(")"):
                args.append(self.expr())
                while self.accept(","):
                    args.append(self.expr())
                self.take("op", ")")
            return ("launch", kname, grid, block, shm, tuple(args))
        raise ParseError(f"unexpected {kw!r} in host code")

    def hblock(self):
        self.take("op", "{")
        body = []
        while not self.accept("}"):
            st = self.host()
            if st[0] not in ("free", "launch", "hif"):
                raise ParseError(f"{st[0]} inside a host branch")
            body.append(st)
        return tuple(body)

    def block(self):
        self.take("op", "{")
        body = []
        while not self.accept("}"):
            body.append(self.kstmt())
        return tuple(body)

    def kstmt(self):
        kw = self.take("kw")
        if kw == "let":
            name = self.take("name")
            self.take("op", "=")
            return ("let", name, self.expr())
        if kw in ("shared", "local"):
            name = self.take("name")
            self.take("op", "[")
            size = self.expr()
            self.take("op", "]")
            return ("static", name, size)
        if kw == "dynshared":
            return ("dynshared", self.take("name"))
        if kw == "partition":
            name = self.take("name")
            self.take("op", "=")
            base = self.take("name")
            self.take("op", "+")
            return ("partition", name, base, self.expr())
        if kw == "free":
            return ("free", self.take("name"))
        if kw in ("load", "store", "atomic"):
            ds = self.take("name")
            self.take("op", "[")
            idx = self.expr()
            self.take("op", "]")
            return ("access", kw, ds, idx)
        if kw == "if":
            self.take("op", "(")
            c = self.expr()
            self.take("op", ")")
            then = self.block()
            other = self.block() if self.accept("else") else ()
            return ("if", c, then, other)
        if kw == "guard":
            return ("guard", self.expr())
        if kw == "for":
            v = self.take("name")
            self.take("op", "<")
            bound = self.expr()
            return ("for", v, bound, self.block())
        raise ParseError(f"unexpected {kw!r} in kernel code")

    def program(self):
        host, kernels = [], {}
        while self.peek()[0] != "eof":
            if self.peek() == ("kw", "kernel"):
                self.take()
                name = self.take("name")
                self.take("op", "(")
                params = []
                if not self.accept(")"):
                    params.append(self.take("name"))
                    while self.accept(","):
                        params.append(self.take("name"))
                    self.take("op", ")")
                if name in kernels:
                    raise ParseError(f"kernel {name} defined twice")
                kernels[name] = (tuple(params), self.block())
            else:
                host.append(self.host())
        return tuple(host), kernels


@dataclass
class Program:
    """A parsed program: host statements in order and kernels by name."""
    text: str
    host: tuple
    kernels: dict
    name: str = ""
    widths: dict = field(default_factory=dict)    # input name -> bits

    @property
    def input_names(self):
        return [s[1] for s in self.host if s[0] == "input"]

    def accesses(self, kernel: str):
        """The memory instructions of a kernel in program order:
        (index, op, data structure)."""
        out = []

        def walk(body):
            for s in body:
                if s[0] == "access":
                    out.append((len(out), s[1], s[2]))
                elif s[0] == "if":
                    walk(s[2])
                    walk(s[3])
                elif s[0] == "for":
                    walk(s[3])
        walk(self.kernels[kernel][1])
        return out

    def launches(self):
        """Launch statements in program order (then-branches first)."""
        out = []

        def walk(stmts):
            for s in stmts:
                if s[0] == "launch":
                    out.append(s)
                elif s[0] == "hif":
                    walk(s[2])
                    walk(s[3])
        walk(self.host)
        return out


def _names_in(e, out):
    if e[0] == "ref":
        out.add(e[1])
    elif e[0] == "bin":
        _names_in(e[2], out)
        _names_in(e[3], out)
    elif e[0] == "not":
        _names_in(e[1], out)
    return out


def _check_types(e, want: str, where: str) -> None:
    """Comparisons and ``&& || !`` are boolean, the rest integer; ``/``,
    ``%`` and ``<<`` take an integer literal on the right (positive for the
    first two)."""
    if e[0] in ("num", "ref"):
        got = "int"
    elif e[0] == "not":
        _check_types(e[1], "bool", where)
        got = "bool"
    else:
        op, a, b = e[1], e[2], e[3]
        if op in ("&&", "||"):
            _check_types(a, "bool", where)
            _check_types(b, "bool", where)
            got = "bool"
        else:
            _check_types(a, "int", where)
            _check_types(b, "int", where)
            if op in ("/", "%", "<<") and (b[0] != "num" or (op != "<<" and b[1] == 0)):
                raise ParseError(f"{where}: {op} needs a {'positive ' if op != '<<' else ''}literal on the right")
            got = "int" if op in ("+", "-", "*", "/", "%", "<<") else "bool"
    if got != want:
        raise ParseError(f"{where}: {expr_text(e)} is {got}, {want} expected")


def parse(text: str, name: str = "") -> Program:
    """Parse and check scoping: every name is defined once, before its use;
    kernel parameters are bound by the launches; partitions and static arrays
    sit at the top level of their kernel, partitions of a dynamic shared base."""
    host, kernels = _Parser(text).program()
    widths, defined, ptrs = {}, set(), set()

    def use(e, scope):
        for n in _names_in(e, set()):
            if n not in scope and n not in BUILTINS:
                raise ParseError(f"{name}: {n} used before its definition")
    def host_stmts(stmts):
        for s in stmts:
            if s[0] == "hif":
                use(s[1], defined)
                _check_types(s[1], "bool", name)
                yield s
                yield from host_stmts(s[2])
                yield from host_stmts(s[3])
            else:
                yield s
    for s in host_stmts(host):
        if s[0] == "hif":
            continue
        if s[0] == "free":
            if s[1] not in ptrs:
                raise ParseError(f"{name}: free of {s[1]}, not a malloc'd buffer")
            continue
        if s[0] in ("input", "let", "malloc"):
            if s[1] in defined:
                raise ParseError(f"{name}: {s[1]} defined twice")
            if s[0] == "input":
                if not 1 <= s[2] <= 64:
                    raise ParseError(f"{name}: input {s[1]} needs 1..64 bits")
                widths[s[1]] = s[2]
            else:
                use(s[2], defined)
                _check_types(s[2], "int", name)
                if s[0] == "malloc":
                    ptrs.add(s[1])
            defined.add(s[1])
        elif s[0] == "assert":
            use(s[1], defined)
            _check_types(s[1], "bool", name)
        else:
            _, kname, grid, block, shm, args = s
            if kname not in kernels:
                raise ParseError(f"{name}: launch of unknown kernel {kname}")
            if len(args) != len(kernels[kname][0]):
                raise ParseError(f"{name}: {kname} takes {len(kernels[kname][0])} arguments")
            for e in grid + block + args + ((shm,) if shm else ()):
                use(e, defined)
                _check_types(e, "int", name)
            for e in grid + block + ((shm,) if shm else ()):
                if any(n in ptrs for n in _names_in(e, set())) or _names_in(e, set()) & set(BUILTINS):
                    raise ParseError(f"{name}: launch dimensions use a pointer or a builtin")
    for kname, (params, body) in kernels.items():
        scope = set(params)
        if len(scope) != len(params):
            raise ParseError(f"{name}: repeated parameter in {kname}")

        def walk(body, top):
            for s in body:
                k = s[0]
                if k in ("let", "static", "dynshared", "partition", "for"):
                    nm = s[1]
                    if nm in scope:
                        raise ParseError(f"{name}: {nm} defined twice in {kname}")
                if k in ("static", "dynshared", "partition") and not top:
                    raise ParseError(f"{name}: {k} {s[1]} must be at the top level of {kname}")
                if k in ("static", "dynshared", "partition") and seen_access:
                    raise ParseError(f"{name}: {k} {s[1]} must precede the accesses of {kname}")
                if k == "access":
                    seen_access.append(s)
                if k == "free":
                    if s[1] not in params:
                        raise ParseError(f"{name}: free of {s[1]}, not a parameter of {kname}")
                elif k == "let":
                    use(s[2], scope)
                    _check_types(s[2], "int", name)
                elif k == "static":
                    if _names_in(s[2], set()):
                        raise ParseError(f"{name}: static array {s[1]} needs a constant size")
                    _check_types(s[2], "int", name)
                elif k == "partition":
                    use(s[3], scope)
                    _check_types(s[3], "int", name)
                    if s[2] not in dyn:
                        raise ParseError(f"{name}: partition {s[1]} of {s[2]}, not a dynamic shared base")
                elif k == "access":
                    if s[2] not in scope:
                        raise ParseError(f"{name}: access to unknown {s[2]}")
                    use(s[3], scope)
                    _check_types(s[3], "int", name)
                elif k == "if":
                    use(s[1], scope)
                    _check_types(s[1], "bool", name)
                    walk(s[2], False)
                    walk(s[3], False)
                elif k == "guard":
                    use(s[1], scope)
                    _check_types(s[1], "bool", name)
                elif k == "for":
                    use(s[2], scope)
                    _check_types(s[2], "int", name)
                    scope.add(s[1])
                    walk(s[3], False)
                    continue
                if k in ("let", "static", "dynshared", "partition"):
                    scope.add(s[1])
                if k == "dynshared":
                    if dyn:
                        raise ParseError(f"{name}: {kname} has two dynamic shared bases")
                    dyn.add(s[1])
        dyn, seen_access = set(), []
        walk(body, True)
    return Program(text=text, host=host, kernels=kernels, name=name, widths=widths)


# ----------------------------------------------------------------- printing
def expr_text(e) -> str:
    if e[0] == "num":
        return str(e[1])
    if e[0] == "ref":
        return e[1]
    if e[0] == "not":
        return f"!({expr_text(e[1])})"
    return f"({expr_text(e[2])} {e[1]} {expr_text(e[3])})"


# ------------------------------------------------------------ example programs
# Hand-written programs in the style of the paper's motivating examples:
# an input-dependent grid over a global buffer (Sec. 2), a dynamic shared
# buffer carved into parts whose sizes come from a kernel argument (Sec. 4.2
# and Fig. 9b), tiles staged through static shared memory, and a strided loop.
EXAMPLES = {
    # grid rounded up to whole blocks; the first kernel guards the index, the
    # second guards it off by one
    "guarded_grid": """
        input n : 8
        malloc A = n
        launch scale grid((n + 31) / 32) block(32) args(A, n)
        launch scale_le grid((n + 31) / 32) block(32) args(A, n)
        kernel scale(p, len) {
          let i = blockIdx.x * blockDim.x + threadIdx.x
          guard i < len
          load p[i]
          store p[i]
        }
        kernel scale_le(p, len) {
          let i = blockIdx.x * blockDim.x + threadIdx.x
          if (i <= len) { store p[i] }
        }
    """,
    # a size that the host asserts to be a multiple of the block: the guard
    # can be dropped safely only under the assert
    "asserted_multiple": """
        input n : 7
        assert n % 16 == 0
        malloc A = n
        malloc B = n + 8
        launch copy grid(n / 16) block(16) args(A, B)
        kernel copy(a, b) {
          let i = blockIdx.x * 16 + threadIdx.x
          load a[i]
          store b[i + 8]
          store b[i + 9]
        }
    """,
    # dynamic shared memory in three parts: keys (m entries), values (m
    # entries), then a scratch tail; thread t touches keys[t], values[t] and
    # values[t + 1] (the last reaches into the tail, or past the end)
    "shm_partitions": """
        input m : 5
        input extra : 3
        malloc A = m
        launch kv grid(1) block(m) shm(2 * m + extra) args(A, m)
        kernel kv(p, len) {
          dynshared base
          partition vals = base + len
          partition tail = base + 2 * len
          let t = threadIdx.x
          load base[t]
          store vals[t]
          store vals[t + 1]
          load tail[t]
          load p[t]
        }
    """,
    # a 2-D tile staged through static shared memory with a halo of one
    "tile_halo": """
        input w : 4
        input h : 4
        malloc img = w * h
        launch blur grid(1, 1) block(w, h) args(img, w)
        kernel blur(p, ld) {
          shared tile[240]
          let x = threadIdx.x
          let y = threadIdx.y
          store tile[y * 16 + x]
          store tile[(y + 1) * 16 + x]
          load p[y * ld + x]
          if (x + 1 < ld) { load p[y * ld + x + 1] } else { load p[y * ld + x - 1] }
        }
    """,
    # a per-thread loop over one row; the store is shifted by one, so the
    # last row's last iteration writes one past the end of B
    "strided_loop": """
        input n : 6
        input k : 3
        assert k >= 1
        malloc A = n * k
        malloc B = n * k
        launch rows grid(2) block(4) args(A, B, n, k)
        kernel rows(a, b, len, per) {
          local acc[4]
          let row = blockIdx.x * 4 + threadIdx.x
          guard row < len
          for j < per {
            load a[row * per + j]
            store b[row * per + j + 1]
          }
          store acc[threadIdx.x]
        }
    """,
    # a stencil that reads one element to the left: a lower-bound access
    "stencil_left": """
        input n : 6
        malloc A = n + 1
        launch left grid(1) block(n) args(A)
        kernel left(p) {
          let i = threadIdx.x
          load p[i - 1]
          if (i >= 1) { store p[i - 1] }
        }
    """,
}


def examples():
    return [parse(t, name) for name, t in EXAMPLES.items()]


# ------------------------------------------------------------ random programs
def random_program(rng: np.random.Generator, name: str = "") -> Program:
    """One small program with one or two inputs of 3-4 bits, a launch of at
    most 4 x 8 threads, and accesses to a global buffer, a static shared
    array and parts of the dynamic shared buffer, each behind a guard drawn
    from correct, off-by-one and missing.  Small enough that every input and
    every thread can be enumerated."""
    r = lambda n: int(rng.integers(n))
    wn, wm = 3 + r(2), 2 + r(2)
    bdim = [4, 8][r(2)]
    scale = 1 + r(3)
    pad = r(3)
    lines = [f"input n : {wn}", f"input m : {wm}"]
    lines.append(f"malloc A = n * {scale} + {pad}")
    if r(2):
        lines.append("assert n >= m")
    grid = [f"(n + {bdim - 1}) / {bdim}", "2", "m + 1"][r(3)]
    shm = f"m + {r(4)}"
    lines.append(f"launch k grid({grid}) block({bdim}) shm({shm}) args(A, n, m)")
    guard_i = ["i < len", "i <= len", "i < len + 1", None][r(4)]
    body = ["let i = blockIdx.x * blockDim.x + threadIdx.x"]
    static = [bdim, bdim + 1, bdim - 1][r(3)]
    body.append(f"shared s[{static}]")
    body.append("dynshared base")
    part = ["half", None][r(2)]
    if part:
        body.append("partition half = base + cnt / 2")
    g_off = [f"i * {scale}", f"i * {scale} + {pad}", f"i * {scale} + {scale - 1}"][r(3)]
    if guard_i:
        body.append(f"if ({guard_i}) {{ load p[{g_off}] }}")
    else:
        body.append(f"load p[{g_off}]")
    body.append(["store s[threadIdx.x]", "store s[threadIdx.x + 1]",
                 "if (threadIdx.x >= 1) { store s[threadIdx.x - 1] }"][r(3)])
    t_guard = ["threadIdx.x < cnt", "threadIdx.x <= cnt", "threadIdx.x < cnt / 2"][r(3)]
    if part:
        body.append(f"if ({t_guard}) {{ load base[threadIdx.x] }}")
        body.append(f"if ({t_guard}) {{ store half[threadIdx.x] }}")
    else:
        body.append(f"if ({t_guard}) {{ load base[threadIdx.x] }} else {{ atomic base[0] }}")
    if r(2):
        body.append(f"for j < cnt {{ load p[j * {scale}] }}")
    kern = "kernel k(p, len, cnt) {\n  " + "\n  ".join(body) + "\n}"
    return parse("\n".join(lines) + "\n" + kern, name)


def random_programs(seed: int = 11, n: int = 24):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_program(rng, f"rprog{seed}_{i}") for i in range(n)]


# --------------------------------------------------- use-after-free programs
UAF_EXAMPLES = {
    # a buffer freed on one path, then passed to a launch; then freed for good
    "free_then_launch": """
        input c : 1
        malloc A = 8
        malloc B = 8
        launch k grid(1) block(4) args(A, B)
        if (c == 1) { free A }
        launch k grid(1) block(4) args(A, B)
        free B
        launch k grid(1) block(4) args(A, B)
        kernel k(p, q) { load p[threadIdx.x] store q[threadIdx.x] }
    """,
    # device-side frees: one under a branch before a later read, one at the
    # end of a loop body before the next iteration's read
    "device_free": """
        input n : 2
        input f : 1
        malloc A = 4
        malloc B = 4
        launch k grid(1) block(2) args(A, B, n, f)
        kernel k(p, q, cnt, flag) {
          shared s[2]
          load p[0]
          if (flag == 1) { free p }
          store s[threadIdx.x]
          for j < cnt {
            load q[j]
            if (flag == 0) { free q }
          }
          load p[1]
        }
    """,
    # two branches on the same condition: the buffer is never used after its
    # free in any run, but a path-insensitive analysis pairs the free of one
    # branch with the launch of the other
    "correlated_branches": """
        input c : 1
        malloc A = 4
        if (c == 1) { free A }
        if (c == 0) { launch k grid(1) block(1) args(A) }
        kernel k(p) { load p[0] }
    """,
}


def uaf_examples():
    return [parse(t, name) for name, t in UAF_EXAMPLES.items()]


def random_uaf_program(rng: np.random.Generator, name: str = "") -> Program:
    """Host code with two buffers (A of n + 1 elements, B of 4), frees and
    launches under branches that each test an input of their own (so every
    path is feasible), and a kernel whose device frees sit under branches on
    a flag argument before unconditional accesses and loops of up to n
    iterations."""
    r = lambda n: int(rng.integers(n))
    n_if = 2 + r(3)
    lines = [f"input c{i} : 1" for i in range(n_if)]
    lines += ["input n : 2", "input f : 1", "malloc A = n + 1", "malloc B = 4"]
    launch = "launch k grid(1) block(2) args(A, B, n, f)"
    lines.append(launch)
    for i in range(n_if):
        lines.append([f"if (c{i} == 1) {{ free A }}", f"if (c{i} == 1) {{ free B }}",
                      f"if (c{i} == 1) {{ free A }} else {{ free B }}",
                      f"if (c{i} == 1) {{ {launch} }}",
                      f"if (c{i} == 1) {{ {launch} }} else {{ free A }}"][r(5)])
        if r(2):
            lines.append(launch)
    body = ["load p[0]"]
    for t in range(1 + r(3)):
        body.append(["if (flag == 1) { free p }", "if (flag == 0) { free q }", "load p[1]",
                     "store q[0]", f"for j{t} < cnt {{ load q[j{t}] if (flag == 1) {{ free q }} }}",
                     f"for j{t} < cnt {{ store p[j{t}] }}"][r(6)])
    kern = "kernel k(p, q, cnt, flag) {\n  " + "\n  ".join(body) + "\n}"
    return parse("\n".join(lines) + "\n" + kern, name)


def random_uaf_programs(seed: int = 21, n: int = 64):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_uaf_program(rng, f"ruaf{seed}_{i}") for i in range(n)]
