"""Concrete interpreter of the small GPU programs: TEST INFRASTRUCTURE ONLY.

It answers, by running the program, the question that the front-end's
queries ask symbolically (paper Sec. 4.1 and Sec. 5.2): can this memory
instruction, in this launch, touch an element outside its data structure?
The host code runs statement by statement for one assignment of the inputs
(an assert that fails ends the run, as the program would abort); every launch
runs every thread of its grid (blocks and threads on three axes) through the
kernel body, with loops iterated and guards taken as written.  An access is
out of bounds above when its offset is at least the size of its data
structure, below when the offset is negative.

Sizes of data structures: a global buffer has the size its ``malloc`` gave;
a static array its declared size; the dynamic shared buffer is split at the
partition offsets in program order, each part ending where the next begins
and the last one at the dynamic shared size of the launch (the layout that
Sec. 4.2 and Fig. 9b describe).

Use after free (paper Sec. 4.3 and Sec. 5.3): the run also tracks which
buffers are live.  On the host a ``malloc`` makes a buffer live and a
``free`` ends it; a launch that passes a buffer that is not live is a use
after free, reported as ``("uaf", "launch", launch index, kernel, argument
position)``.  In a kernel every parameter and every array is live when the
thread starts, a device ``free`` ends the parameter for the rest of that
thread, and an access to a data structure that is not live is reported as
``("uaf", "access", kernel, access index)``.

``brute_force`` enumerates every input assignment, which is the plain
definition of "some legal input makes the access go out of bounds"; it is
meant for programs of a few input bits and a few hundred threads.
Arithmetic is exact (Python integers); ``/`` and ``%`` of a negative value
raise, as the program format leaves them undefined.
"""
from __future__ import annotations

import itertools

AX = "xyz"


class ProgramError(ValueError):
    pass


def _value(e, env):
    t = e[0]
    if t == "num":
        return e[1]
    if t == "ref":
        v = env[e[1]]
        if isinstance(v, tuple):
            raise ProgramError(f"pointer {e[1]} used as a value")
        return v
    if t == "not":
        return not _value(e[1], env)
    op, a = e[1], _value(e[2], env)
    if op == "&&":
        return bool(a) and bool(_value(e[3], env))
    if op == "||":
        return bool(a) or bool(_value(e[3], env))
    b = _value(e[3], env)
    if op == "+":
        return a + b
    if op == "-":
        return a - b
    if op == "*":
        return a * b
    if op in ("/", "%"):
        if a < 0:
            raise ProgramError("division of a negative value")
        return a // b if op == "/" else a % b
    if op == "<<":
        return a * 2 ** b
    return {"<": a < b, "<=": a <= b, ">": a > b, ">=": a >= b, "==": a == b, "!=": a != b}[op]


def _number_accesses(body, out):
    """Program-order index of every access statement (then-branch before
    else-branch, loop bodies in place)."""
    for s in body:
        if s[0] == "access":
            out[id(s)] = len(out)
        elif s[0] == "if":
            _number_accesses(s[2], out)
            _number_accesses(s[3], out)
        elif s[0] == "for":
            _number_accesses(s[3], out)
    return out


class _Thread:
    def __init__(self, kname, li, numbering, sizes, shm, record, params):
        self.kname, self.li, self.num = kname, li, numbering
        self.sizes = dict(sizes)          # buffer name -> size (globals filled in)
        self.shm = shm
        self.parts = []                   # [(name, offset)] of the dynamic shared buffer
        self.record = record
        self.loops = {}
        self.live = set(params)           # data structures this thread may still use

    def part_size(self, name):
        names = [p[0] for p in self.parts]
        j = names.index(name)
        end = self.parts[j + 1][1] if j + 1 < len(self.parts) else self.shm
        return end - self.parts[j][1]

    def block(self, stmts, env):
        for s in stmts:
            k = s[0]
            if k == "let":
                env[s[1]] = _value(s[2], env)
            elif k == "static":
                self.sizes[s[1]] = _value(s[2], env)
                self.live.add(s[1])
            elif k == "dynshared":
                self.parts.append((s[1], 0))
                self.live.add(s[1])
            elif k == "partition":
                self.parts.append((s[1], _value(s[3], env)))
                self.live.add(s[1])
            elif k == "free":
                self.live.discard(s[1])
            elif k == "access":
                ds = s[2]
                offset = _value(s[3], env)
                size = self.sizes[ds] if ds in self.sizes else self.part_size(ds)
                ai = self.num[id(s)]
                if ds not in self.live:
                    self.record(("uaf", "access", self.kname, ai), env, dict(self.loops))
                if offset >= size:
                    self.record((self.li, self.kname, ai, "upper"), env, dict(self.loops))
                if offset < 0:
                    self.record((self.li, self.kname, ai, "lower"), env, dict(self.loops))
            elif k == "if":
                self.block(s[2] if _value(s[1], env) else s[3], env)
            elif k == "guard":
                if not _value(s[1], env):
                    return
            elif k == "for":
                for v in range(max(_value(s[2], env), 0)):
                    env[s[1]] = v
                    self.loops[s[1]] = v
                    self.block(s[3], env)
                self.loops.pop(s[1], None)
                env.pop(s[1], None)


def _number_launches(stmts, out):
    """Program-order index of every launch statement, then-branches of host
    ``if`` blocks before their else-branches."""
    for s in stmts:
        if s[0] == "launch":
            out[id(s)] = len(out)
        elif s[0] == "hif":
            _number_launches(s[2], out)
            _number_launches(s[3], out)
    return out


class _Abort(Exception):
    pass


def run(prog, inputs: dict, record, only=None):
    """Run the program for one input assignment; ``record(key, env, loops)``
    is called for every out-of-bounds access.  ``only`` = (launch index,
    block (x, y, z), thread (x, y, z)) runs just that thread of that launch.
    Returns False when an assert stopped the run."""
    env = {}
    sizes = {}
    numbering = _number_launches(prog.host, {})
    try:
        _host(prog, prog.host, inputs, env, sizes, numbering, record, only, set())
    except _Abort:
        return False
    return True


def _host(prog, stmts, inputs, env, sizes, launch_no, record, only, live):
    for s in stmts:
        k = s[0]
        if k == "input":
            env[s[1]] = inputs[s[1]]
        elif k == "let":
            env[s[1]] = _value(s[2], env)
        elif k == "malloc":
            sizes[s[1]] = _value(s[2], env)
            env[s[1]] = ("ptr", s[1])
            live.add(s[1])
        elif k == "free":
            live.discard(s[1])
        elif k == "assert":
            if not _value(s[1], env):
                raise _Abort()
        elif k == "hif":
            _host(prog, s[2] if _value(s[1], env) else s[3], inputs, env, sizes, launch_no, record,
                  only, live)
        elif k == "launch":
            li = launch_no[id(s)]
            _, kname, grid, blk, shm, args = s
            if only is not None and only[0] != li:
                continue
            g = [_value(e, env) for e in grid]
            b = [_value(e, env) for e in blk]
            shm_v = _value(shm, env) if shm is not None else 0
            params, body = prog.kernels[kname]
            kenv0, ksizes = {}, {}
            for pos, (name, a) in enumerate(zip(params, args)):
                if a[0] == "ref" and isinstance(env[a[1]], tuple):
                    ksizes[name] = sizes[a[1]]
                    if a[1] not in live and only is None:
                        record(("uaf", "launch", li, kname, pos), env, {})
                else:
                    kenv0[name] = _value(a, env)
            numbering = _number_accesses(body, {})
            if only is not None:
                blocks, threads = [only[1]], [only[2]]
                if not all(0 <= only[1][i] < g[i] and 0 <= only[2][i] < b[i] for i in range(3)):
                    continue
            else:
                blocks = [(x, y, z) for z in range(max(g[2], 0)) for y in range(max(g[1], 0))
                          for x in range(max(g[0], 0))]
                threads = [(x, y, z) for z in range(max(b[2], 0)) for y in range(max(b[1], 0))
                           for x in range(max(b[0], 0))]
            for bid in blocks:
                for tid in threads:
                    kenv = dict(kenv0)
                    for i, a in enumerate(AX):
                        kenv[f"threadIdx.{a}"] = tid[i]
                        kenv[f"blockIdx.{a}"] = bid[i]
                        kenv[f"blockDim.{a}"] = b[i]
                        kenv[f"gridDim.{a}"] = g[i]
                    _Thread(kname, li, numbering, ksizes, shm_v, record, params).block(body, kenv)
    return True


def keys(prog, lower=True):
    """Every (launch index, kernel, access index, bound) of the program."""
    out = []
    launches = []

    def walk(stmts):
        for s in stmts:
            if s[0] == "launch":
                launches.append(s)
            elif s[0] == "hif":
                walk(s[2])
                walk(s[3])
    walk(prog.host)
    for li, s in enumerate(launches):
        n = len(_number_accesses(prog.kernels[s[1]][1], {}))
        for ai in range(n):
            out.append((li, s[1], ai, "upper"))
            if lower:
                out.append((li, s[1], ai, "lower"))
    return out


def brute_force(prog, lower=True):
    """key -> (out of bounds for some input?, first witness, number of
    (input, thread, iteration) events).  A witness is (inputs, block,
    thread, loop counters)."""
    res = {k: [False, None, 0] for k in keys(prog, lower)}
    names = [s[1] for s in prog.host if s[0] == "input"]
    widths = [s[2] for s in prog.host if s[0] == "input"]
    for vals in itertools.product(*[range(2 ** w) for w in widths]):
        inputs = dict(zip(names, vals))

        def record(key, env, loops):
            if key not in res:
                return
            r = res[key]
            if not r[0]:
                bid = tuple(env[f"blockIdx.{a}"] for a in AX)
                tid = tuple(env[f"threadIdx.{a}"] for a in AX)
                r[0], r[1] = True, (dict(inputs), bid, tid, loops)
            r[2] += 1
        run(prog, inputs, record)
    return {k: tuple(v) for k, v in res.items()}


def witness_goes_out(prog, key, values: dict) -> bool:
    """True iff the assignment ``values`` (input names, ``threadIdx.x`` ...,
    ``blockIdx.x`` ..., ``for:<counter>``; absent names are 0) makes the
    access ``key`` go out of bounds in that thread, at those loop counters."""
    names = [s[1] for s in prog.host if s[0] == "input"]
    inputs = {n: int(values.get(n, 0)) for n in names}
    bid = tuple(int(values.get(f"blockIdx.{a}", 0)) for a in AX)
    tid = tuple(int(values.get(f"threadIdx.{a}", 0)) for a in AX)
    want = {k[4:]: int(v) for k, v in values.items() if k.startswith("for:")}
    hits = []

    def record(k, env, loops):
        if k == key and all(loops.get(n) == v for n, v in want.items()):
            hits.append(loops)
    run(prog, inputs, record, only=(key[0], bid, tid))
    return bool(hits)


def uaf_brute_force(prog):
    """Every use after free that some input assignment makes happen: the
    set of ``("uaf", ...)`` keys met over all runs."""
    found = set()
    names = [s[1] for s in prog.host if s[0] == "input"]
    widths = [s[2] for s in prog.host if s[0] == "input"]
    for vals in itertools.product(*[range(2 ** w) for w in widths]):
        def record(key, env, loops):
            if key[0] == "uaf":
                found.add(key)
        run(prog, dict(zip(names, vals)), record)
    return found
