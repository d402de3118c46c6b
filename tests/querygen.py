"""Random small query DAGs for exhaustive tests (test helper, no arithmetic
of its own: it only builds DAGs with the workloads builder)."""
import numpy as np

from workloads import Query


def random_query(rng: np.random.Generator, max_bits: int = 10, n_ops: int = 6,
                 ops=("add", "sub", "mul", "shl", "udiv", "urem", "const"),
                 name: str = "") -> Query:
    q = Query(name or "rand")
    nv = int(rng.integers(1, 4))
    widths = []
    for i in range(nv):
        w = int(rng.integers(1, 4))
        if sum(widths) + w > max_bits:
            break
        widths.append(w)
    ints = [q.var(f"x{i}", w) for i, w in enumerate(widths)]
    nonneg = list(ints)            # nodes known to be >= 0 (for udiv/urem)
    for _ in range(n_ops):
        op = ops[int(rng.integers(len(ops)))]
        a = ints[int(rng.integers(len(ints)))]
        b = ints[int(rng.integers(len(ints)))]
        if op == "add":
            e = a + b
            if a in nonneg and b in nonneg:
                nonneg.append(e)
        elif op == "sub":
            e = a - b
        elif op == "mul":
            e = a * b
            if a in nonneg and b in nonneg:
                nonneg.append(e)
        elif op == "shl":
            e = a << int(rng.integers(0, 3))
            if a in nonneg:
                nonneg.append(e)
        elif op in ("udiv", "urem"):
            a = nonneg[int(rng.integers(len(nonneg)))]
            k = int(rng.integers(1, 6))
            e = a // k if op == "udiv" else a % k
            nonneg.append(e)
        else:
            e = q.const(int(rng.integers(0, 9)))
            nonneg.append(e)
        ints.append(e)
    n_roots = int(rng.integers(1, 4))
    for _ in range(n_roots):
        a = ints[int(rng.integers(len(ints)))]
        b = ints[int(rng.integers(len(ints)))]
        kind = int(rng.integers(0, 9))
        c = [a < b, a <= b, a > b, a >= b, a.eq(b), a.ne(b)][kind % 6]
        if kind == 6:
            c = ~c
        elif kind == 7:
            c = c | (ints[0] < ints[-1])
        elif kind == 8:
            c = c & (ints[-1] >= ints[0])
        q.require(c)
    return q
