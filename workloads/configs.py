"""Seeded generators for the OOB-query workloads.

Each generator returns ``GenQuery`` records: the query, the verdict it has
by construction, and for SAT queries an input assignment the construction
makes out-of-bounds (checked by the oracle's exact integer evaluator in the
tests, never trusted blindly).

The shapes follow the relations the paper shows: a 1-D global thread index
bounded by the launch (saxpy, Fig. 5; Sec. 4.1), guards that dominate the
access (the ``if (i < numv)`` of Fig. 2), sizes and offsets in bytes for
``cudaMalloc`` buffers, and partitions of one allocation at prefix-sum
offsets with sizes by subtraction (Fig. 9b; Sec. 5.1).  Inputs are unsigned
and arithmetic is exact (no wrap-around).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .query import Query

SAT, UNSAT = "SAT", "UNSAT"


@dataclass
class GenQuery:
    query: Query
    label: str                       # verdict by construction
    witness: dict = field(default_factory=dict)   # var name -> value (SAT)
    kind: str = ""


def oob_1d(width: int, guard: str, scale: int = 4, header: int = 0,
           name: str = "") -> Query:
    """One global access ``buf[idx]`` with ``idx = blockIdx*blockDim +
    threadIdx`` into a buffer of ``N`` elements of ``scale`` bytes after a
    ``header``-byte prefix.

    guard: ``"lt"`` (idx < N), ``"le"`` (idx <= N, off by one) or
    ``"none"``.  Constraint kinds (Sec. 5.2): threadIdx < blockDim (kind 1),
    offset and size defined by their trees (kind 3), offset >= size (kind 2).
    """
    q = Query(name or f"oob1d_w{width}_{guard}_s{scale}_c{header}")
    N = q.var("N", width)
    bdim = q.var("blockDim", width)
    bid = q.var("blockIdx", width)
    tid = q.var("threadIdx", width)
    q.require(tid < bdim)
    idx = bid * bdim + tid
    if guard == "lt":
        q.require(idx < N)
    elif guard == "le":
        q.require(idx <= N)
    else:
        assert guard == "none"
    if header:
        offset = idx * scale + header
        size = N * scale + header
    else:
        offset = idx * scale
        size = N * scale
    q.require(offset >= size)
    return q


def config1(variant: str = "lt") -> GenQuery:
    """The single query: 12-bit N, blockDim, blockIdx, threadIdx; guard
    idx < N; size 4*N bytes; offset 4*idx; OOB test offset >= size."""
    q = oob_1d(12, variant, scale=4, header=0, name=f"config1_{variant}")
    if variant == "lt":
        return GenQuery(q, UNSAT, kind="guarded")
    if variant == "none":
        return GenQuery(q, SAT, dict(N=0, blockDim=1, blockIdx=0, threadIdx=0),
                        kind="unguarded")
    return GenQuery(q, SAT, dict(N=1, blockDim=1, blockIdx=1, threadIdx=0),
                    kind="off_by_one")


def config2(seed: int = 2, n: int = 256, wmin: int = 8, wmax: int = 16):
    """Batch of 1-D queries: widths w ~ U{wmin..wmax}; element size s in
    {1,2,4,8}; header c ~ U{0..16}; half with the correct guard (UNSAT),
    a quarter unguarded and a quarter off by one (SAT); shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ["lt"] * (n // 2) + ["none"] * (n // 4)
    kinds += ["le"] * (n - len(kinds))
    kinds = [kinds[i] for i in rng.permutation(n)]
    out = []
    for i, g in enumerate(kinds):
        w = int(rng.integers(wmin, wmax + 1))
        s = int(rng.choice([1, 2, 4, 8]))
        c = int(rng.integers(0, 17))
        q = oob_1d(w, g, scale=s, header=c, name=f"c2_{i}_w{w}_{g}_s{s}_c{c}")
        if g == "lt":
            out.append(GenQuery(q, UNSAT, kind="guarded"))
        elif g == "none":
            out.append(GenQuery(q, SAT, dict(N=0, blockDim=1, blockIdx=0,
                                             threadIdx=0), kind="unguarded"))
        else:
            out.append(GenQuery(q, SAT, dict(N=1, blockDim=2, blockIdx=0,
                                             threadIdx=1), kind="off_by_one"))
    return out


def partition_query(width: int, lens_w: int, k_sub: int, target: int,
                    index: str, guard: str, level: str = "partition",
                    name: str = "") -> Query:
    """Accesses into partition ``target`` of one allocation split into
    ``k_sub`` parts (Sec. 4.2; Fig. 9b).  Part i starts at the prefix sum of
    the lengths before it; the size of a part is the next start minus its
    own start, and the last part's size is the allocation size minus its
    start.  Units are elements.

    index: ``"t"`` (idx = t) or ``"tw"`` (idx = t*W + i with i < W).
    guard: ``"lt"`` (idx < len_target), ``"le"`` (idx <= len_target), or
    ``"next"`` / ``"prev"`` (guard against a neighbour's length).
    level: ``"partition"`` tests idx >= size(part); ``"allocation"`` tests
    start(part) + idx >= S.
    """
    q = Query(name or f"part_k{k_sub}_j{target}_{index}_{guard}_{level}")
    lens = [q.var(f"len{i}", lens_w) for i in range(k_sub)]
    for ln in lens:
        q.require(ln >= 1)                       # assert len_i >= 1
    S = q.var("S", width)
    total = lens[0]
    for ln in lens[1:]:
        total = total + ln
    q.require(S.eq(total))                       # allocation = sum of parts
    starts = [q.const(0)]
    for i in range(1, k_sub):
        starts.append(starts[-1] + lens[i - 1])
    sizes = [starts[i + 1] - starts[i] for i in range(k_sub - 1)]
    sizes.append(S - starts[-1])
    t = q.var("t", width)
    if index == "t":
        idx = t
    else:
        W = q.var("W", width)
        i_ = q.var("i", width)
        q.require(i_ < W)
        idx = t * W + i_
    bound = {"lt": lens[target], "le": lens[target],
             "next": lens[(target + 1) % k_sub],
             "prev": lens[(target - 1) % k_sub]}[guard]
    if guard == "le":
        q.require(idx <= bound)
    else:
        q.require(idx < bound)
    if level == "partition":
        q.require(idx >= sizes[target])
    else:
        q.require(starts[target] + idx >= S)
    return q


def config5(seed: int = 5, n: int = 1024, width: int = 20):
    """Intra-allocation partition queries: one allocation of `width`-bit
    size split into k_sub ~ U{2..8} parts at prefix-sum offsets, partition
    sizes by subtraction, a guarded access into part j ~ U{0..k_sub-1}.
    Half use the correct guard idx < len_j (UNSAT); half are buggy: idx <=
    len_j (the one-past-the-end index), or a guard against a neighbour's
    length (SAT).  Index idx = t, or t*W + i with i < W."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    kinds = ["lt"] * (n // 2) + ["bug"] * (n - n // 2)
    kinds = [kinds[i] for i in rng.permutation(n)]
    for qi, kind in enumerate(kinds):
        k_sub = int(rng.integers(2, 9))
        j = int(rng.integers(0, k_sub))
        index = "t" if rng.integers(2) == 0 else "tw"
        if kind == "lt":
            guard = "lt"
        else:
            guard = ["le", "next", "prev"][int(rng.integers(3))]
        q = partition_query(width, width, k_sub, j, index, guard, level="partition",
                            name=f"c5_{qi}_k{k_sub}_j{j}_{index}_{guard}")
        if guard == "lt":
            out.append(GenQuery(q, UNSAT, kind="partition_guarded"))
            continue
        # a witness by construction: every part holds one element, except
        # that a neighbour guard's part holds three; the index is one past
        # the end of part j, which the buggy guard still admits
        lens = [1] * k_sub
        if guard != "le":
            lens[(j + 1) % k_sub if guard == "next" else (j - 1) % k_sub] = 3
        idx = 1
        wit = {f"len{i}": lens[i] for i in range(k_sub)}
        wit["S"] = sum(lens)
        if index == "t":
            wit["t"] = idx
        else:
            wit.update(t=idx, W=1, i=0)
        out.append(GenQuery(q, SAT, wit, kind=f"partition_{guard}"))
    return out
