"""Parity of the GPU path (C ABI -> gfx950 kernels) with the CPU oracle.

* COUNT mode: for every cube, the device's (refuted, f, m, count of
  satisfying assignments of the active variables, smallest satisfying
  index) equals the oracle's canonical leaf, bit for bit; over a complete
  cube set the counts add up to the oracle's #DPLL model count.
* DECIDE mode: verdicts equal the oracle's (and the generators' labels);
  every SAT witness satisfies the original query under exact integers.
"""
import numpy as np
import pytest

from oracle import cnf_ref, query_ref
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _raw(ctx, cnfs):
    return ctx.cnf_from_arrays(*w.concat(cnfs))


def _check_leaves(cnfs, cubes_per_query, out, complete=True, kinds=None):
    for qi, (f, cubes) in enumerate(zip(cnfs, cubes_per_query)):
        total = 0
        for c, cube in enumerate(cubes):
            lf = out.leaf(qi, c)
            ref = cnf_ref.leaf(f, cube)
            if kinds is not None and kinds[qi][c] == 2:
                # pruned by backjumping: not evaluated, and it has no model
                assert lf["refuted"] and (ref["refuted"] or ref["count"] == 0)
                continue
            assert lf["refuted"] == ref["refuted"], (f.name, c, cube, lf, ref)
            if ref["refuted"]:
                continue
            got = (lf["f"], lf["m"], lf["count"], lf["first"])
            want = (ref["f"], ref["m"], ref["count"], ref["first"])
            assert got == want, (f.name, c, cube, got, want)
            total += lf["count"] << lf["m"]
        if complete:
            assert total == cnf_ref.count(f), f.name


LEAF_VARIANTS = ["scalar", "vector", "lds"]


@pytest.mark.parametrize("leaf", LEAF_VARIANTS)
def test_count_mode_split_cubes(ctx, leaf):
    """Every leaf of complete splits (k = 8, 14, 20: one block to 256
    blocks of 4096 assignments) under each leaf-evaluation variant."""
    rng = np.random.Generator(np.random.PCG64(101))
    cnfs = []
    for n, ratio in ((24, 3.0), (30, 4.26), (40, 4.26), (48, 3.5), (36, 2.0), (60, 4.26)):
        cnfs.append(w.random_ksat(n, int(round(ratio * n)), 3, rng))
    raw = _raw(ctx, cnfs)
    for k in (8, 14, 20):
        cubes = ctx.split(raw, k=k)
        out = ctx.solve(raw, cubes, mode=1, leaf=leaf)
        per_q = [cubes.view(i)["cubes"] for i in range(len(cnfs))]
        kinds = [cubes.view(i)["kind"] for i in range(len(cnfs))]
        for i in range(len(cnfs)):
            assert cubes.view(i)["complete"]
        _check_leaves(cnfs, per_q, out, kinds=kinds)


def test_count_mode_oracle_cubes(ctx):
    """Cubes drawn on the test side (random partial assignments, some of
    them clashing), not by the library's splitter."""
    rng = np.random.Generator(np.random.PCG64(102))
    cnfs, cubes = [], []
    for n in (16, 20, 26, 33):
        f = w.random_ksat(n, int(round(3.8 * n)), 3, rng)
        cnfs.append(f)
        qc = [[]]
        for _ in range(12):
            size = int(rng.integers(0, n // 2))
            vs = rng.choice(n, size=size, replace=False) + 1
            qc.append([int(v) if rng.integers(2) else -int(v) for v in vs])
        v = int(rng.integers(1, n + 1))
        qc.append([v, -v])                       # a clashing cube
        cubes.append(qc)
    raw = _raw(ctx, cnfs)
    cb = ctx.cubes_from_arrays(raw, cubes)
    out = ctx.solve(raw, cb, mode=1)
    _check_leaves(cnfs, cubes, out, complete=False)


@pytest.mark.parametrize("pigeons,holes,want", [(3, 3, 6), (4, 4, 24), (5, 5, 120),
                                                (5, 4, 0), (6, 5, 0)])
def test_pigeonhole_single_leaf(ctx, pigeons, holes, want):
    f = w.pigeonhole(pigeons, holes)
    raw = _raw(ctx, [f])
    cubes = ctx.cubes_from_arrays(raw, [[[]]])
    out = ctx.solve(raw, cubes, mode=1)
    lf = out.leaf(0, 0)
    assert not lf["refuted"] and lf["f"] == pigeons * holes
    assert lf["count"] << lf["m"] == want


def test_degenerate_formulas(ctx):
    cnfs = [w.CNF.from_clauses(3, []),                 # no clauses: SAT, 8 models
            w.CNF.from_clauses(2, [[1], []]),          # empty clause: UNSAT
            w.CNF.from_clauses(4, [[1], [-1, 2]]),     # decided by propagation
            w.CNF.from_clauses(5, [[1, 2], [-1, -2]]),  # f = 2 < 6
            w.CNF.from_clauses(9, [[1, 2, 3], [4, 5, 6], [7, 8, 9], [-1, -4, -7]])]  # 6 < f < 12
    raw = _raw(ctx, cnfs)
    cubes = ctx.split(raw, k=20)
    out = ctx.solve(raw, cubes, mode=1)
    per_q = [cubes.view(i)["cubes"] for i in range(len(cnfs))]
    _check_leaves(cnfs, per_q, out, kinds=[cubes.view(i)["kind"] for i in range(len(cnfs))])
    dec = ctx.decide(raw, k=20)
    assert dec.verdicts() == ["SAT", "UNSAT", "SAT", "SAT", "SAT"]


def test_product_cnf_counts_small_widths(ctx):
    """Model counts of the library's own CNFs (split + COUNT leaves) equal
    the number of satisfying input tuples by brute force."""
    from tests.querygen import random_query
    rng = np.random.Generator(np.random.PCG64(103))
    qs = [random_query(rng, max_bits=10, name=f"r{i}") for i in range(40)]
    qs += [w.oob_1d(3, g, scale=s, header=c) for g in ("lt", "le", "none")
           for (s, c) in ((1, 0), (4, 3))]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs])
    cubes = ctx.split(cnf, k=14)
    out = ctx.solve(cnf, cubes, mode=1)
    for i, q in enumerate(qs):
        cv = cubes.view(i)
        assert cv["complete"]
        total = 0
        for c in range(len(cv["cubes"])):
            lf = out.leaf(i, c)
            if not lf["refuted"]:
                total += lf["count"] << lf["m"]
        assert total == query_ref.int_bruteforce(q)[1], q.name


def test_decide_single_access(ctx):
    gens = [w.single_access("lt"), w.single_access("none"), w.single_access("le")]
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label
        if g.label == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))


@pytest.mark.parametrize("opts", [
    dict(k=30),                                             # the library's defaults
    dict(k=30, leaves_per_round=1, chunk_log2=12),          # the launch point bench.py times
    dict(k=30, leaves_per_round=1, chunk_log2=12, scorer="word"),
    dict(k=30, leaves_per_round=1, chunk_log2=12, leaf="vector"),
    dict(k=30, leaves_per_round=1, chunk_log2=12, leaf="lds"),
], ids=["defaults", "bench_point", "word", "leaf_vector", "leaf_lds"])
def test_decide_batch_1d_full(ctx, opts):
    gens = w.batch_1d()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, **opts)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label, (g.query.name, r)
        ov, _, _ = query_ref.decide(g.query)
        assert ov == r["verdict"], g.query.name
        if g.label == "SAT":
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))


def test_decide_small_queries_brute_force(ctx):
    from tests.querygen import random_query
    rng = np.random.Generator(np.random.PCG64(104))
    qs = [random_query(rng, max_bits=12, name=f"d{i}") for i in range(60)]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs])
    for k in (6, 16):
        res = ctx.decide(cnf, k=k, leaves_per_round=2)
        for i, q in enumerate(qs):
            want = query_ref.int_bruteforce(q)[0]
            r = res.result(i)
            assert r["verdict"] == want, (q.name, k, r)
            if want == "SAT":
                assert query_ref.int_eval(q, res.witness(i, q.n_vars))


def test_decide_lower_bound_batch(ctx):
    """256 lower-bound stencil reads (offset < 0 with signed exact
    arithmetic): verdicts equal the labels and the oracle's, and every
    witness reads below the buffer under exact integers."""
    gens = w.batch_lower()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, leaves_per_round=1, chunk_log2=12)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label, (g.query.name, r)
        assert query_ref.decide(g.query)[0] == r["verdict"], g.query.name
        if g.label == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))


def test_decide_wrap32_batch(ctx):
    """256 guarded accesses with 32-bit machine integers (SCUBA_BB_WRAP(32)).
    Those whose byte size N*s can wrap are found SAT, with a witness that
    goes out of bounds under 32-bit arithmetic.  The others are refuted at
    the root: the guard bounds the (possibly wrapping) index, so index and
    size times s cannot wrap, and the exact root check applies."""
    from paper_2601_21552_amd import _lib
    gens = w.batch_wrap(m=32)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens], flags=_lib.BB_WRAP(32))
    res = ctx.decide(cnf, k=30, leaves_per_round=1, chunk_log2=12, max_cubes=300)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] in (g.label, "UNKNOWN"), (g.query.name, r)
        if g.label == "SAT":
            assert r["verdict"] == "SAT", g.query.name
            assert r["witness_checked"]
            assert query_ref.wrap_eval(g.query, res.witness(i, g.query.n_vars), 32)
        else:
            assert r["verdict"] == "UNSAT" and r["how"] == "root", g.query.name


@pytest.mark.parametrize("m", [4, 6])
def test_decide_wrap_small_brute_force(ctx, m):
    from paper_2601_21552_amd import _lib
    from tests.querygen import random_query
    rng = np.random.Generator(np.random.PCG64(501 + m))
    qs = [random_query(rng, max_bits=10, name=f"wd{m}_{i}") for i in range(60)]
    qs = [q for q in qs if max(q.var_widths) <= m]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs], flags=_lib.BB_WRAP(m))
    for k in (4, 12):
        res = ctx.decide(cnf, k=k, leaves_per_round=2)
        for i, q in enumerate(qs):
            want = query_ref.wrap_bruteforce(q, m)[0]
            r = res.result(i)
            assert r["verdict"] == want, (q.name, k, r)
            if want == "SAT":
                assert query_ref.wrap_eval(q, res.witness(i, q.n_vars), m)


def _witness_values(g):
    """Generator witness as input values in declaration order."""
    return [g.witness[name] for name in g.query.var_names]


def test_decide_partition_batch(ctx):
    """1024 intra-allocation partition queries (20-bit sizes, 2..8 parts)
    under the word ordering: every guarded access UNSAT at the root, every
    buggy one SAT with a witness that goes past its partition under exact
    integers; the oracle's verdict on a sample (DPLL, else the generator's
    witness checked by the definition)."""
    gens = w.partition_batch()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, max_cubes=20000, scorer="word")
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label, (g.query.name, r)
        if g.label == "UNSAT":
            assert query_ref.root_check(g.query) == "UNSAT"
        else:
            assert r["witness_checked"]
            wit = res.witness(i, g.query.n_vars)
            assert query_ref.int_eval(g.query, wit), g.query.name
            if i % 16 == 0:
                ov, _, how = query_ref.decide(g.query, max_nodes=300, candidate=_witness_values(g))
                assert ov == "SAT", (g.query.name, how)


def test_decide_partition_batch_static_never_wrong(ctx):
    """The static most-occurrences ordering on the same queries: UNKNOWN
    when its walk runs out of cubes (the case the word ordering and the
    learned scorer address), never a wrong verdict."""
    gens = w.partition_batch()[:256]
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, max_cubes=3000)
    for i, g in enumerate(gens):
        r = res.result(i)
        if g.label == "SAT" and r["verdict"] == "UNKNOWN":
            continue
        assert r["verdict"] == g.label, (g.query.name, r)
        if g.label == "SAT":
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))


def test_decide_batch_2d_one_call(ctx):
    """All 4096 2-D accesses of uneven width (8..24 bits, 1..3 multipliers)
    in one decide call: labels reproduced, correct ones UNSAT by the root
    relaxation (the oracle's own root check agrees), every SAT witness
    verified under exact integers."""
    gens = w.batch_2d()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, max_cubes=20000, scorer="word")
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label, (g.query.name, r)
        if g.label == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars)), g.query.name
        elif i % 8 == 0:
            assert query_ref.root_check(g.query) == "UNSAT", g.query.name


def _component_cnf(nv, rng, name):
    """Variables 1..nv split into components of 2-4 variables, each with 1-3
    random clauses of 2-3 literals over its own variables, every variable in
    some clause.  Components share no variable, so the model count is the
    product of the components' counts and the smallest satisfying index
    (slot j = variable j + 1, all variables active) is the sum of each
    component's smallest contribution; both are found by enumerating each
    component's few assignments: closed forms that need no search."""
    perm = rng.permutation(nv) + 1
    comps, i = [], 0
    while i < nv:
        size = int(rng.integers(2, 5))
        if nv - i - size == 1:
            size += 1
        comps.append(sorted(int(v) for v in perm[i:i + size]))
        i += size
    clauses, count, first = [], 1, 0
    for vs in comps:
        while True:
            cl = []
            for _ in range(int(rng.integers(1, 4))):
                k = int(rng.integers(2, min(3, len(vs)) + 1))
                pick = rng.choice(vs, size=k, replace=False)
                cl.append([int(v) if rng.integers(2) else -int(v) for v in pick])
            if {abs(l) for c in cl for l in c} == set(vs):
                break
        clauses += cl
        sols = []
        for bits in range(1 << len(vs)):
            val = {v: (bits >> t) & 1 for t, v in enumerate(vs)}
            if all(any((val[abs(l)] == 1) == (l > 0) for l in c) for c in cl):
                sols.append(sum(val[v] << (v - 1) for v in vs))
        count *= len(sols)
        first += min(sols)
    return w.CNF.from_clauses(nv, clauses, name=name), count, first


@pytest.mark.parametrize("leaf", LEAF_VARIANTS)
@pytest.mark.parametrize("f", [31, 34, 38])
def test_count_high_slots_closed_form(ctx, f, leaf):
    """Leaves of 31..38 active variables reach the block-index slots 12..37
    (block bits up to 25): COUNT over one whole-formula leaf equals the
    closed-form count and smallest satisfying index."""
    rng = np.random.Generator(np.random.PCG64(700 + f))
    cnf, count, first = _component_cnf(f, rng, f"comp{f}")
    raw = _raw(ctx, [cnf])
    cubes = ctx.cubes_from_arrays(raw, [[[]]])
    out = ctx.solve(raw, cubes, mode=1, chunk_log2=12, leaf=leaf)
    lf = out.leaf(0, 0)
    assert (lf["refuted"], lf["f"], lf["m"]) == (False, f, 0), lf
    assert lf["count"] == count and lf["first"] == first, (lf, count, first)


def _word_ops_reference(f, cube):
    """The leaf evaluation's word operations of one leaf with at most 12
    active variables (one block of 4096 assignments, no block-level
    literals), reproduced on the CPU in the kernel's fixed order: residual
    clauses in clause order, four at a time, the block abandoned after the
    first group that leaves no assignment alive.  Every evaluated clause
    costs 64 words x (|c| + 1)."""
    ref = cnf_ref.leaf(f, cube)
    if ref["refuted"]:
        return 0
    conflict, assign = cnf_ref.up(f, cube)
    slots = {v: j for j, v in enumerate(ref["slots"])}
    a = np.arange(4096, dtype=np.int64)
    alive = a < (1 << ref["f"])
    res = []
    for cl in f.clauses():
        if any((assign[abs(l)] == 1) == (l > 0) for l in cl if assign[abs(l)] >= 0):
            continue
        res.append([l for l in cl if assign[abs(l)] < 0])
    ops = 0
    for g in range(0, len(res), 4):
        for cl in res[g:g + 4]:
            sat = np.zeros(4096, dtype=bool)
            for l in cl:
                bit = (a >> slots[abs(l)]) & 1
                sat |= (bit == 1) if l > 0 else (bit == 0)
            alive &= sat
            ops += 64 * (len(cl) + 1)
        if not alive.any():
            break
    return ops


@pytest.mark.parametrize("leaf", LEAF_VARIANTS)
def test_word_ops_counter_reproduced(ctx, leaf):
    """The leaf kernel's count of algorithmic word operations equals the
    CPU's replay of its fixed evaluation order on one-block leaves (each
    variant tests for a dead block after every fourth clause it evaluates
    and at the end of the clauses, which on a one-block leaf, where every
    clause is evaluated, is the replay's rule)."""
    rng = np.random.Generator(np.random.PCG64(103))
    cnfs, cubes = [], []
    for n in (14, 18, 22, 26):
        f = w.random_ksat(n, int(round(4.0 * n)), 3, rng)
        cnfs.append(f)
        qc = []
        for _ in range(10):
            vs = rng.choice(n, size=n - 10, replace=False) + 1
            qc.append([int(v) if rng.integers(2) else -int(v) for v in vs])
        cubes.append(qc)
    raw = _raw(ctx, cnfs)
    out = ctx.solve(raw, ctx.cubes_from_arrays(raw, cubes), mode=1, leaf=leaf)
    for qi, (f, qc) in enumerate(zip(cnfs, cubes)):
        want = sum(_word_ops_reference(f, c) for c in qc)
        assert out.result(qi)["word_ops"] == want, (qi, out.result(qi)["word_ops"], want)
