"""Host-side checks of the library (no GPU): every declared entry point is
exported, the CNF of every query has exactly one model per satisfying input
tuple (against brute force), malformed input is rejected, and the cube
splitter's trees are complete and disjoint with leaves matching the
oracle's canonical leaves."""
import re
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

from oracle import cnf_ref, query_ref
from tests.querygen import random_query
import workloads as w
from workloads import CNF, Query


@pytest.fixture(scope="module")
def api():
    from paper_2601_21552_amd import _lib, api as api_mod
    import os
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2601_21552_amd import build
        build.build()
    return api_mod


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _cnf(view):
    return CNF(view["n_vars"], view["clause_off"], view["lits"])


def test_every_declared_symbol_is_exported(api):
    import ctypes
    from paper_2601_21552_amd import _lib
    with open(_lib.os.path.join(_lib.HERE, "..", "include", "scuba.h")) as f:
        header = f.read()
    declared = set(re.findall(
        r"^(?:scuba_status|void|const char\*|uint32_t|size_t)\s+(scuba_[a-z_0-9]+)\s*\(", header, re.M))
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(_lib.SIGNATURES), declared ^ set(_lib.SIGNATURES)
    assert _lib.load().scuba_abi_version() == 1


@pytest.mark.parametrize("flags", [0, 1])
def test_cnf_counts_equal_integer_solutions(ctx, flags):
    rng = np.random.Generator(np.random.PCG64(201 + flags))
    qs = [random_query(rng, max_bits=9, name=f"r{i}") for i in range(80)]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs], flags=flags)
    for i, q in enumerate(qs):
        v = cnf.view(i)
        assert cnf_ref.count(_cnf(v)) == query_ref.int_bruteforce(q)[1], q.nodes


@pytest.mark.parametrize("m", [3, 4, 6])
def test_wrap_cnf_counts_equal_machine_solutions(ctx, m):
    """With m-bit machine integers (SCUBA_BB_WRAP(m)) the library's CNF has
    one model per input tuple that satisfies the query under m-bit
    arithmetic: the oracle's model count of that CNF equals exhaustive
    search with the same arithmetic."""
    from paper_2601_21552_amd import _lib
    rng = np.random.Generator(np.random.PCG64(301 + m))
    qs = [random_query(rng, max_bits=8, name=f"m{m}_{i}") for i in range(60)]
    qs = [q for q in qs if max(q.var_widths) <= m]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs], flags=_lib.BB_WRAP(m))
    for i, q in enumerate(qs):
        v = cnf.view(i)
        want = query_ref.wrap_bruteforce(q, m)[1]
        if v["root_unsat"]:   # refuted by the no-wrap abstraction: no m-bit model
            assert want == 0, q.nodes
        else:
            assert cnf_ref.count(_cnf(v)) == want, q.nodes


@pytest.mark.parametrize("m", [3, 4, 5, 6])
def test_wrap_root_refutation_is_sound(ctx, m):
    """Machine-integer queries refuted at the root (arithmetic that cannot
    wrap kept exact, the rest abstracted, then the exact root check) have no
    satisfying input tuple under m-bit arithmetic, by exhaustive search; and
    the refutation does happen on guarded accesses that cannot wrap."""
    from paper_2601_21552_amd import _lib
    rng = np.random.Generator(np.random.PCG64(911 + m))
    qs = [random_query(rng, max_bits=9, n_ops=8, name=f"s{m}_{i}") for i in range(300)]
    qs = [q for q in qs if max(q.var_widths) <= m]
    # guarded accesses idx*s >= N*s under idx < N, with and without room
    # for N*s in m bits (the bit-level pins of these shapes are in the
    # oracle tests)
    for wd in range(1, m + 1):
        for s_ in (1, 2, 4):
            qs.append(w.oob_1d(wd, "lt", scale=s_, header=0, name=f"g{m}_{wd}_{s_}"))
    qs = [q for q in qs if sum(q.var_widths) <= 16]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs], flags=_lib.BB_WRAP(m))
    refuted = 0
    for i, q in enumerate(qs):
        if cnf.view(i)["root_unsat"]:
            refuted += 1
            assert query_ref.wrap_bruteforce(q, m)[0] == "UNSAT", (m, q.name, q.nodes)
    assert refuted > 0


def test_wrap_batch_refuted_at_the_root(ctx):
    """In the 32-bit batch every guarded access whose size cannot wrap is
    refuted at the root (its label is pinned by the oracle tests) and no
    access whose size wraps is."""
    from paper_2601_21552_amd import _lib
    gens = w.batch_wrap(m=32)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens], flags=_lib.BB_WRAP(32))
    for i, g in enumerate(gens):
        assert bool(cnf.view(i)["root_unsat"]) == (g.label == "UNSAT"), g.query.name


def test_wrap_rejects_inputs_wider_than_the_machine_word(api, ctx):
    from paper_2601_21552_amd import _lib
    q = Query("wide")
    x = q.var("x", 40)
    q.require(x > 3)
    assert _status(api, lambda: ctx.bitblast([q.arrays()[:2]], flags=_lib.BB_WRAP(32))) == -2   # SCUBA_E_WIDTH


def test_packed_batch_gives_the_same_cnf(api, ctx):
    gens = w.batch_1d(n=32) + [w.single_access("none")]
    arrays = [g.query.arrays()[:2] for g in gens]
    a = ctx.bitblast(arrays)
    b = ctx.bitblast_packed(*api.pack_queries(arrays))
    assert len(a) == len(b) == len(gens)
    for i in range(len(gens)):
        va, vb = a.view(i), b.view(i)
        assert va["n_vars"] == vb["n_vars"] and va["root_unsat"] == vb["root_unsat"]
        assert np.array_equal(va["clause_off"], vb["clause_off"])
        assert np.array_equal(va["lits"], vb["lits"])
    assert len(ctx.bitblast_packed(*api.pack_queries([]))) == 0


def test_input_map_and_witness_decoding(ctx):
    g = w.single_access("none")
    cnf = ctx.bitblast([g.query.arrays()[:2]])
    first, width = cnf.input_map(0)
    assert list(width) == [12, 12, 12, 12]
    assert list(first) == [1, 13, 25, 37]          # inputs take the first variables
    v = cnf.view(0)
    verdict, model, _ = cnf_ref.solve(_cnf(v))
    assert verdict == "SAT"
    vals = [sum(int(model[f + b]) << b for b in range(wd)) for f, wd in zip(first, width)]
    assert query_ref.int_eval(g.query, vals)


def test_root_unsat_on_guarded_queries(ctx):
    gens = w.batch_1d()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    for i, g in enumerate(gens):
        assert cnf.view(i)["root_unsat"] == (g.label == "UNSAT"), g.query.name
    one = ctx.bitblast([w.single_access("lt").query.arrays()[:2]]).view(0)
    assert one["root_unsat"] and one["n_clauses"] == 1


def test_root_unsat_on_lower_bound_queries(ctx):
    """Guarded lower-bound reads (idx >= h, offset (idx - h)*s < 0) are
    decided at the root; the off-by-one and unguarded ones are not."""
    gens = w.batch_lower()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    for i, g in enumerate(gens):
        assert cnf.view(i)["root_unsat"] == (g.label == "UNSAT"), g.query.name


def test_root_unsat_on_2d_queries(ctx):
    """The library's relaxation with product lemmas decides every correct
    2-D access at the root and never a buggy one."""
    gens = w.batch_2d(n=400)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    for i, g in enumerate(gens):
        assert cnf.view(i)["root_unsat"] == (g.label == "UNSAT"), g.query.name


def _status(api, fn):
    from paper_2601_21552_amd import _lib
    with pytest.raises(_lib.ScubaError) as e:
        fn()
    return e.value.status


def test_malformed_queries_are_rejected(api, ctx):
    q = Query("wide")
    q.var("x", 8)
    nodes, roots, _ = q.arrays()
    bad = nodes.copy()
    bad["width"][0] = 65
    assert _status(api, lambda: ctx.bitblast([(bad, np.array([0], np.uint32))])) == -2
    q = Query("fwd")
    x = q.var("x", 4)
    q.require(x < 3)
    nodes, roots, _ = q.arrays()
    fwd = nodes.copy()
    fwd["a"][-1] = len(fwd)                      # operand after the node
    assert _status(api, lambda: ctx.bitblast([(fwd, roots)])) == -1
    # an integer node as a root
    assert _status(api, lambda: ctx.bitblast([(nodes, np.array([0], np.uint32))])) == -1
    # division of a value that can be negative
    q = Query("negdiv")
    x, y = q.var("x", 3), q.var("y", 3)
    q.require(((x - y) // 2) < 1)
    assert _status(api, lambda: ctx.bitblast([q.arrays()[:2]])) == -1


def test_raw_cnf_validation(api, ctx):
    ok = ctx.cnf_from_arrays([3], [0, 2], [0, 2, 3], [1, -2, 3])
    assert ok.view(0)["n_clauses"] == 2
    rep = lambda: ctx.cnf_from_arrays([3], [0, 1], [0, 2], [1, -1])
    assert _status(api, rep) == -1
    rng = lambda: ctx.cnf_from_arrays([3], [0, 1], [0, 1], [4])
    assert _status(api, rng) == -1


def _kraft_and_disjoint(cubes):
    total = sum(Fraction(1, 2 ** len(c)) for c in cubes)
    assert total == 1
    for a, b in combinations(cubes, 2):
        sa = set(a)
        assert any(-l in sa for l in b), (a, b)


def test_split_trees_complete_disjoint_and_canonical(ctx):
    rng = np.random.Generator(np.random.PCG64(202))
    cnfs = [w.random_ksat(n, int(r * n), 3, rng) for n, r in ((14, 4.3), (18, 3.0), (22, 4.26))]
    cnfs.append(w.pigeonhole(4, 3))
    cnfs.append(w.pigeonhole(5, 4))     # backjumping prunes here
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    for k in (3, 7, 12):
        cubes = ctx.split(raw, k=k)
        for i, f in enumerate(cnfs):
            cv = cubes.view(i)
            assert cv["complete"]
            _kraft_and_disjoint(cv["cubes"])
            total = 0
            for c, cube in enumerate(cv["cubes"]):
                ref = cnf_ref.leaf(f, cube)
                if cv["kind"][c] == 1:
                    assert ref["refuted"]
                elif cv["kind"][c] == 2:      # pruned by backjumping: no model
                    assert ref["refuted"] or ref["count"] == 0
                else:
                    assert not ref["refuted"] and ref["f"] == cv["f"][c] <= k
                    total += ref["count"] << ref["m"]
            assert total == cnf_ref.count(f)


def test_word_order_trees_count_integer_solutions(ctx):
    """Word ordering on bit-blasted queries: complete, disjoint trees whose
    leaf counts add up to the number of integer solutions."""
    rng = np.random.Generator(np.random.PCG64(203))
    qs = [random_query(rng, max_bits=10, name=f"wo{i}") for i in range(30)]
    qs += [w.oob_2d(2, g, 1, 2, 1, False) for g in ("no_row", "col_le", "ld_free")]
    cnf = ctx.bitblast([q.arrays()[:2] for q in qs])
    for k in (2, 6):
        cubes = ctx.split(cnf, k=k, scorer="word")
        static = ctx.split(cnf, k=k)
        differ = False
        for i, q in enumerate(qs):
            cv = cubes.view(i)
            assert cv["complete"]
            _kraft_and_disjoint(cv["cubes"])
            differ |= cv["cubes"] != static.view(i)["cubes"]
            v = cnf.view(i)
            f = CNF(v["n_vars"], v["clause_off"], v["lits"])
            total = 0
            for c, cube in enumerate(cv["cubes"]):
                if cv["kind"][c] != 0:
                    continue
                ref = cnf_ref.leaf(f, cube)
                assert not ref["refuted"] and ref["f"] == cv["f"][c] <= k
                total += ref["count"] << ref["m"]
            assert total == query_ref.int_bruteforce(q)[1], q.name
        assert differ


def test_split_budget_marks_incomplete(ctx):
    g = w.single_access("none")
    cnf = ctx.bitblast([g.query.arrays()[:2]])
    cv = ctx.split(cnf, k=20, max_cubes=10).view(0)
    assert not cv["complete"] and len(cv["cubes"]) == 10


def test_decide_needs_a_device(api, ctx):
    """Without a GPU the device entry points fail loudly (no CPU fallback)."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cnf = ctx.bitblast([w.single_access("none").query.arrays()[:2]])
    from paper_2601_21552_amd import _lib
    with pytest.raises(Exception):
        ctx.decide(cnf, k=30)
    assert _lib.load() is not None


def _active_count(cnf, assign):
    """Unassigned variables occurring in a clause that no literal satisfies."""
    act = set()
    for c in range(cnf.n_clauses):
        lits = cnf.lits[cnf.clause_off[c]:cnf.clause_off[c + 1]]
        if any((l > 0 and assign[l] == 1) or (l < 0 and assign[-l] == 0) for l in lits):
            continue
        act.update(abs(int(l)) for l in lits if assign[abs(l)] < 0)
    return len(act)


def test_trace_root_labels_match_lookahead(api, ctx):
    """Rows of the root node: the candidates are the first active variables of
    the static order (most literal occurrences, ties to the lowest index) and
    each label is log2(1 + f - f0) + log2(1 + f - f1), with f0 / f1 the active
    counts after propagating the variable to 0 / 1 (0 on a conflict)."""
    rng = np.random.Generator(np.random.PCG64(77))
    cnfs = [w.random_ksat(36, 150, 3, rng) for _ in range(4)]
    batch = ctx.cnf_from_arrays(*w.concat(cnfs))
    m = 6
    feats, labels, nodes = ctx.trace(batch, k=6, candidates=m, every=1, depth=64)
    assert feats.shape == (len(labels), 16) and len(nodes) == len(labels)
    for qi, c in enumerate(cnfs):
        sel = nodes == ((qi << 32) | 1)
        conflict, a = cnf_ref.up(c)
        assert not conflict
        f = _active_count(c, a)
        occ = np.zeros(c.n_vars + 1, np.int64)
        np.add.at(occ, np.abs(c.lits), 1)
        active = {abs(int(l)) for j in range(c.n_clauses)
                  for l in c.lits[c.clause_off[j]:c.clause_off[j + 1]]
                  if a[abs(l)] < 0}
        order = sorted(range(1, c.n_vars + 1), key=lambda v: (-occ[v], v))
        cands = [v for v in order if v in active][:m]
        assert sel.sum() == len(cands)
        want = []
        for v in cands:
            fb = []
            for lit in (-v, v):
                cf, ab = cnf_ref.up(c, [lit])
                fb.append(0 if cf else _active_count(c, ab))
            want.append(np.log2(1 + f - fb[0]) + np.log2(1 + f - fb[1]))
        np.testing.assert_allclose(labels[sel], want, rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(feats[sel][:, 6], occ[cands] / 64.0, rtol=1e-6)
        np.testing.assert_allclose(feats[sel][:, 9], f / 256.0, rtol=1e-6)
        assert np.all(feats[sel][:, 15] == 1.0)


def test_learned_options_are_validated(api, ctx):
    from paper_2601_21552_amd import _lib
    rng = np.random.Generator(np.random.PCG64(78))
    c = w.random_ksat(20, 80, 3, rng)
    batch = ctx.cnf_from_arrays(*w.concat([c]))
    bad = _lib.LearnedScorer(None, None, 16, 1)
    with pytest.raises(_lib.ScubaError):
        ctx.decide_workspace(batch, learned=bad)
    ok_ptrs = _lib.LearnedScorer(1 << 20, 1 << 20, 1, 1)   # candidates below 2
    with pytest.raises(_lib.ScubaError):
        ctx.decide_workspace(batch, learned=ok_ptrs)
    assert ctx.lib.scuba_scorer_workspace(batch.h, 16) >= 16 * (16 + 2 * 128) * 2


def test_trace_word_candidates_and_range_label(api, ctx):
    """On a bit-blasted query (encoded as given, so input ranges come from
    the input bits alone) the root's candidates are the first active
    variables of the static order plus the most significant active bit of
    each input word, and each label adds the reduction of the inputs'
    range width in bits, sum of log2(hi - lo + 1), over the two branches."""
    from paper_2601_21552_amd import _lib
    q = w.oob_1d(4, "none", scale=2, header=1)
    batch = ctx.bitblast([q.arrays()[:2]], flags=_lib.BB_NO_REWRITE)
    v = batch.view(0)
    c = CNF(v["n_vars"], v["clause_off"], v["lits"])
    first, width = batch.input_map(0)
    first = [int(x) for x in first]
    width = [int(x) for x in width]
    m = 5
    feats, labels, nodes = ctx.trace(batch, k=2, candidates=m, every=1, depth=64)
    sel = nodes == 1
    conflict, a = cnf_ref.up(c)
    assert not conflict

    def active(assign):
        return {abs(int(l)) for j in range(c.n_clauses)
                for l in c.lits[c.clause_off[j]:c.clause_off[j + 1]]
                if assign[abs(l)] < 0
                and not any((x > 0 and assign[x] == 1) or (x < 0 and assign[-x] == 0)
                            for x in c.lits[c.clause_off[j]:c.clause_off[j + 1]])}

    def range_bits(assign):
        bits = 0.0
        for f0, wd in zip(first, width):
            lo = sum(1 << b for b in range(wd) if assign[f0 + b] == 1)
            hi = lo + sum(1 << b for b in range(wd) if assign[f0 + b] < 0)
            bits += np.log2(hi - lo + 1)
        return bits

    act = active(a)
    occ = np.zeros(c.n_vars + 1, np.int64)
    np.add.at(occ, np.abs(c.lits), 1)
    order = sorted(range(1, c.n_vars + 1), key=lambda x: (-occ[x], x))
    cands = [x for x in order if x in act][:m]
    for f0, wd in zip(first, width):
        for b in reversed(range(wd)):
            x = f0 + b
            if a[x] < 0 and x in act:
                if x not in cands:
                    cands.append(x)
                break
    assert sel.sum() == len(cands) > m
    f, r = len(act), range_bits(a)
    want = []
    for x in cands:
        lab = 0.0
        for lit in (-x, x):
            cf, ab = cnf_ref.up(c, [lit])
            lab += np.log2(1 + f - (0 if cf else len(active(ab))))
            lab += r - (0.0 if cf else range_bits(ab))
        want.append(lab)
    np.testing.assert_allclose(labels[sel], want, rtol=1e-4, atol=1e-4)
    # the word candidates are input bits at the top of their words
    tail = feats[sel][m:]
    assert np.all(tail[:, 7] == 1.0)


def test_max_cubes_beyond_witness_key_is_rejected(api):
    """The device witness key holds a cube sequence number below 2^26: a
    larger per-query budget is refused before any work."""
    from paper_2601_21552_amd import _lib
    import workloads as w
    ctx = api.Context(0)
    cnf = ctx.bitblast([w.single_access("lt").query.arrays()[:2]])
    with pytest.raises(_lib.ScubaError):
        ctx.split(cnf, k=30, max_cubes=(1 << 26) + 1)
    with pytest.raises(_lib.ScubaError):
        ctx.decide_workspace(cnf, k=30, max_cubes=(1 << 26) + 1)
    ctx.split(cnf, k=30, max_cubes=1 << 26)


def test_noalloc_rejects_batches_beyond_its_scratch(ctx):
    """The allocation-free decide refuses, before any device work, a batch
    whose workspace bound exceeds its scratch array, and a graph request."""
    import ctypes as C
    from paper_2601_21552_amd import _lib
    from paper_2601_21552_amd.api import _solve_opts
    gens = w.batch_2d(n=256)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    need = ctx.decide_workspace(cnf, k=30)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    h = C.c_void_p()
    st = ctx.lib.scuba_decide_noalloc(ctx.h, cnf.h, C.byref(_solve_opts(k=30)), None, C.byref(h))
    assert st == -5 and not h.value   # SCUBA_E_CAPACITY
    assert "allocation-free" in ctx.lib.scuba_last_error(ctx.h).decode()
    small = ctx.bitblast([g.query.arrays()[:2] for g in w.batch_1d()[:4]])
    st = ctx.lib.scuba_decide_noalloc(ctx.h, small.h, C.byref(_solve_opts(k=30, graph=True)), None,
                                      C.byref(h))
    assert st == -1 and not h.value   # SCUBA_E_INVALID


def test_device_split_options_are_checked(ctx):
    """The device split's option checks run before any device work: no
    graphs, no learned scorer, no given cubes, no allocation-free form, and
    a bounded step; its workspace grows with the step size."""
    import ctypes as C
    from paper_2601_21552_amd import _lib
    from paper_2601_21552_amd.api import _solve_opts
    rng = np.random.Generator(np.random.PCG64(5))
    cnf = ctx.cnf_from_arrays(*w.concat([w.random_ksat(60, 256, 3, rng) for _ in range(8)]))
    small = ctx.decide_workspace(cnf, k=16, device_split=True, split_batch=256)
    big = ctx.decide_workspace(cnf, k=16, device_split=True, split_batch=4096)
    assert 0 < small < big
    for bad in (dict(graph=True), dict(split_batch=(1 << 20) + 1)):
        with pytest.raises(_lib.ScubaError):
            ctx.decide_workspace(cnf, k=16, device_split=True, **bad)
    h = C.c_void_p()
    st = ctx.lib.scuba_decide_noalloc(ctx.h, cnf.h, C.byref(_solve_opts(k=16, device_split=True)), None,
                                      C.byref(h))
    assert st == -1 and not h.value   # SCUBA_E_INVALID
    cubes = ctx.split(cnf, k=16)
    st = ctx.lib.scuba_solve(ctx.h, cnf.h, cubes.h, C.byref(_solve_opts(k=16, device_split=True)),
                             C.c_void_p(1), 1 << 20, None, C.byref(h))
    assert st == -1 and not h.value


def test_tune_cache_round_trip(ctx, tmp_path):
    """The autotuner's cache persists as JSON lines keyed by the device's
    architecture: lines of this device load (a context without a device
    keys them "no-device"), lines of another architecture are skipped, a
    save writes back what was loaded, and a malformed line or options the
    library rejects are errors."""
    import json
    from paper_2601_21552_amd import _lib
    mine = {"gpu": "no-device", "bucket": [11, 8, 2, 1], "k": 20, "chunk_log2": 8, "leaves_per_round": 1,
            "grid": 2048, "scorer": 2, "flags": 5, "max_residual": 4096}
    other = dict(mine, gpu="gfx90a", k=16)
    p = tmp_path / "tune.jsonl"
    p.write_text(json.dumps(mine) + "\n" + json.dumps(other) + "\n")
    assert ctx.tune_cache_load(str(p)) == 1
    out = tmp_path / "saved.jsonl"
    ctx.tune_cache_save(str(out))
    lines = [json.loads(x) for x in out.read_text().splitlines()]
    assert mine in lines and all(x["gpu"] == "no-device" for x in lines)
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"gpu":"no-device","bucket":[1,2,3,4],"k":20}\n')
    with pytest.raises(_lib.ScubaError):
        ctx.tune_cache_load(str(bad))
    bad.write_text(json.dumps(dict(mine, k=50)) + "\n")    # k above the leaf limit of 38
    with pytest.raises(_lib.ScubaError):
        ctx.tune_cache_load(str(bad))
