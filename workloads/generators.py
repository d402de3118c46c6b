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
from .cnf import random_ksat_batch

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


def oob_lower_1d(width: int, guard: str, halo: int, scale: int = 4, name: str = "") -> Query:
    """A stencil read ``buf[idx - halo]`` below the start of its buffer:
    ``idx = blockIdx*blockDim + threadIdx``, byte offset
    ``(idx - halo) * scale`` from the allocation's start, and the lower-bound
    test ``offset < 0`` (the other side of the access range, with exact,
    signed arithmetic).

    guard: ``"ge"`` (idx >= halo), ``"ge_off"`` (idx >= halo - 1, off by
    one) or ``"none"``.
    """
    assert 1 <= halo < 2 ** width
    q = Query(name or f"oobl_w{width}_{guard}_h{halo}_s{scale}")
    bdim = q.var("blockDim", width)
    bid = q.var("blockIdx", width)
    tid = q.var("threadIdx", width)
    q.require(tid < bdim)
    idx = bid * bdim + tid
    if guard == "ge":
        q.require(idx >= halo)
    elif guard == "ge_off":
        q.require(idx + 1 >= halo)
    else:
        assert guard == "none"
    offset = (idx - halo) * scale
    q.require(offset < 0)
    return q


def batch_lower(seed: int = 6, n: int = 256, wmin: int = 8, wmax: int = 16):
    """Batch of lower-bound stencil queries: widths w ~ U{wmin..wmax}, halo
    ~ U{1..8}, element size s in {1,2,4,8}; half guarded (UNSAT), a quarter
    unguarded and a quarter off by one (SAT); shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ["ge"] * (n // 2) + ["none"] * (n // 4)
    kinds += ["ge_off"] * (n - len(kinds))
    kinds = [kinds[i] for i in rng.permutation(n)]
    out = []
    for i, g in enumerate(kinds):
        w = int(rng.integers(wmin, wmax + 1))
        h = int(rng.integers(1, 9))
        s = int(rng.choice([1, 2, 4, 8]))
        q = oob_lower_1d(w, g, h, scale=s, name=f"lo_{i}_w{w}_{g}_h{h}_s{s}")
        if g == "ge":
            out.append(GenQuery(q, UNSAT, kind="lower_guarded"))
        elif g == "none":
            out.append(GenQuery(q, SAT, dict(blockDim=1, blockIdx=0, threadIdx=0), kind="lower_unguarded"))
        else:
            out.append(GenQuery(q, SAT, dict(blockDim=h, blockIdx=0, threadIdx=h - 1),
                                kind="lower_off_by_one"))
    return out


def batch_wrap(seed: int = 7, n: int = 256, m: int = 32, wspan: int = 3):
    """Guarded 1-D accesses (guard idx < N, test idx*s >= N*s) evaluated with
    m-bit machine integers: widths w ~ U{m-wspan..m}, element size s in
    {1,2,4,8}.  The byte size N*s wraps once N >= 2^m / s, which a w-bit N
    reaches iff s * 2^w > 2^m: then N = 2^m / s makes the size 0 and the
    first element is already past it (SAT).  Otherwise no product wraps,
    idx < N gives idx*s < N*s, and the guard holds (UNSAT)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        w = int(rng.integers(max(1, m - wspan), m + 1))
        s = int(rng.choice([1, 2, 4, 8]))
        q = oob_1d(w, "lt", scale=s, header=0, name=f"wr{m}_{i}_w{w}_s{s}")
        if s * (1 << w) > (1 << m):
            out.append(GenQuery(q, SAT, dict(N=(1 << m) // s, blockDim=1, blockIdx=0, threadIdx=0),
                                kind="size_wraps"))
        else:
            out.append(GenQuery(q, UNSAT, kind="no_wrap"))
    return out


def single_access(variant: str = "lt") -> GenQuery:
    """The single query: 12-bit N, blockDim, blockIdx, threadIdx; guard
    idx < N; size 4*N bytes; offset 4*idx; OOB test offset >= size."""
    q = oob_1d(12, variant, scale=4, header=0, name=f"single_{variant}")
    if variant == "lt":
        return GenQuery(q, UNSAT, kind="guarded")
    if variant == "none":
        return GenQuery(q, SAT, dict(N=0, blockDim=1, blockIdx=0, threadIdx=0),
                        kind="unguarded")
    return GenQuery(q, SAT, dict(N=1, blockDim=1, blockIdx=1, threadIdx=0),
                    kind="off_by_one")


def batch_1d(seed: int = 2, n: int = 256, wmin: int = 8, wmax: int = 16):
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
        q = oob_1d(w, g, scale=s, header=c, name=f"b1d_{i}_w{w}_{g}_s{s}_c{c}")
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


def partition_batch(seed: int = 5, n: int = 1024, width: int = 20):
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
                            name=f"part_{qi}_k{k_sub}_j{j}_{index}_{guard}")
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


def oob_2d(width: int, guard: str, mult: int, scale: int, header: int,
           separate_ld: bool, name: str = "") -> Query:
    """A row-major 2-D access ``buf[row*ld + col]`` into ``R`` rows of
    ``ld`` elements of ``scale`` bytes after a ``header``-byte prefix.

    mult (multipliers in the offset): 1: row and col are inputs; 2: row =
    by*bdy + ty with ty < bdy; 3: also col = bx*bdx + tx with tx < bdx.
    separate_ld: ld is its own input (with the assert C <= ld unless the
    guard is "ld_free"); otherwise ld is C.
    guard: "ok" (row < R and col < C), "no_row", "no_col", "row_le"
    (row <= R), "col_le" (col <= C) or "ld_free" (ld independent of C, no
    assert)."""
    q = Query(name or f"oob2d_w{width}_{guard}_m{mult}_s{scale}_c{header}")
    R = q.var("R", width)
    C = q.var("C", width)
    if separate_ld or guard == "ld_free":
        ld = q.var("ld", width)
        if guard != "ld_free":
            q.require(C <= ld)
    else:
        ld = C
    if mult >= 2:
        by, bdy, ty = q.var("by", width), q.var("bdy", width), q.var("ty", width)
        q.require(ty < bdy)
        row = by * bdy + ty
    else:
        row = q.var("row", width)
    if mult >= 3:
        bx, bdx, tx = q.var("bx", width), q.var("bdx", width), q.var("tx", width)
        q.require(tx < bdx)
        col = bx * bdx + tx
    else:
        col = q.var("col", width)
    if guard in ("ok", "no_col", "col_le", "ld_free"):
        q.require(row < R)
    elif guard == "row_le":
        q.require(row <= R)
    if guard in ("ok", "no_row", "row_le", "ld_free"):
        q.require(col < C)
    elif guard == "col_le":
        q.require(col <= C)
    offset = (row * ld + col) * scale + header
    size = R * ld * scale + header
    q.require(offset >= size)
    return q


def _witness_2d(guard: str, mult: int, has_ld: bool) -> dict:
    """Inputs that make the buggy access of oob_2d go one element past the
    end: R = 1 row, and either row = 1 (row guard missing or <=) or col =
    1 with one column (col guard missing or <=), or ld = 1 < C = 2."""
    if guard in ("no_row", "row_le"):
        R, C, ld, row, col = 1, 1, 1, 1, 0
    elif guard in ("no_col", "col_le"):
        R, C, ld, row, col = 1, 1, 1, 0, 1
    else:
        R, C, ld, row, col = 1, 2, 1, 0, 1
    wit = dict(R=R, C=C)
    if has_ld:
        wit["ld"] = ld
    if mult >= 2:
        wit.update(by=row, bdy=1, ty=0)
    else:
        wit["row"] = row
    if mult >= 3:
        wit.update(bx=col, bdx=1, tx=0)
    else:
        wit["col"] = col
    return wit


def batch_2d(seed: int = 3, n: int = 4096, wmin: int = 8, wmax: int = 24):
    """4096 row-major 2-D accesses of uneven size: widths w ~ U{wmin..wmax},
    multipliers per offset mult ~ U{1,2,3}, element size s in {1,2,4,8},
    header c ~ U{0..16}.  Half correct (row < R and col < C; ld is C, or a
    separate ld with C <= ld in a quarter of them): UNSAT.  Half buggy,
    evenly over no row guard, no col guard, row <= R, col <= C and an ld
    independent of C: SAT."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bugs = ["no_row", "no_col", "row_le", "col_le", "ld_free"]
    kinds = ["ok"] * (n // 2) + [bugs[i % 5] for i in range(n - n // 2)]
    kinds = [kinds[i] for i in rng.permutation(n)]
    out = []
    for i, g in enumerate(kinds):
        w = int(rng.integers(wmin, wmax + 1))
        mult = int(rng.integers(1, 4))
        s = int(rng.choice([1, 2, 4, 8]))
        c = int(rng.integers(0, 17))
        sep = g == "ok" and rng.random() < 0.25
        q = oob_2d(w, g, mult, s, c, sep, name=f"b2d_{i}_w{w}_{g}_m{mult}_s{s}_c{c}")
        if g == "ok":
            out.append(GenQuery(q, UNSAT, kind="guarded_2d"))
        else:
            out.append(GenQuery(q, SAT, _witness_2d(g, mult, g == "ld_free"),
                                kind=f"2d_{g}"))
    return out


def random_3sat_sets(seed: int = 4, per_n: int = 2500, ns=(100, 150, 200, 250), ratio: float = 4.26):
    """Uniform random 3-SAT at the threshold: per_n instances for each n,
    m = round(ratio * n) clauses.  Returns {n: [CNF, ...]} (no labels: the
    oracle decides them)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {n: random_ksat_batch(n, int(round(ratio * n)), 3, per_n, rng, prefix=f"r3sat_")
            for n in ns}


def random_3sat_train(seed: int = 40, per_n: int = 1000, ns=(100, 150), ratio: float = 4.26):
    """The scorer's training instances for the random 3-SAT workload: the
    same model from a disjoint seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {n: random_ksat_batch(n, int(round(ratio * n)), 3, per_n, rng, prefix=f"c4t_")
            for n in ns}
