"""Parity of the device-side split (scuba_decide with SCUBA_SOLVE_DEVICE_SPLIT)
with the CPU oracle.

* COUNT mode: the device split's leaves (every leaf of the device tree, in
  emission order) add up to the oracle's exact #DPLL model count,
  sum of count * 2^m, for every formula and several k; each leaf is a
  well-formed leaf (f <= k, count <= 2^f, first set iff count > 0).
* DECIDE mode: verdicts equal the oracle's DPLL verdicts (and the
  generators' labels for access queries); every SAT model satisfies every
  clause (checked here again) and, for access queries, the exact integer
  query.  The host-split path gives the same verdicts.
* Small steps (many pushes and pops per query) give the same results.
"""
import numpy as np
import pytest

from oracle import cnf_ref, query_ref
import workloads as w

pytestmark = pytest.mark.gpu

COUNT = 1


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _raw(ctx, cnfs):
    return ctx.cnf_from_arrays(*w.concat(cnfs))


def _formulas(seed, spec):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [w.random_ksat(n, int(round(ratio * n)), 3, rng) for n, ratio in spec]


def _count_totals(ctx, cnfs, k, **opts):
    res = ctx.decide(_raw(ctx, cnfs), mode=COUNT, k=k, device_split=True, max_cubes=1 << 24, **opts)
    for qi, f in enumerate(cnfs):
        r = res.result(qi)
        total = 0
        for j in range(r["leaves_sent"]):
            lf = res.leaf(qi, j)
            assert not lf["refuted"], (f.name, j, lf)
            assert 0 <= lf["f"] <= k and lf["m"] >= 0, (f.name, j, lf)
            assert lf["count"] <= 1 << lf["f"], (f.name, j, lf)
            assert (lf["first"] >= 0) == (lf["count"] > 0), (f.name, j, lf)
            if lf["first"] >= 0:
                assert lf["first"] < 1 << lf["f"], (f.name, j, lf)
            total += lf["count"] << lf["m"]
        want = cnf_ref.count(f)
        assert total == want, (f.name, k, total, want)
        assert r["verdict"] == ("SAT" if want else "UNSAT"), (f.name, r)
        assert r["cubes_total"] == r["leaves_sent"] + r["cubes_refuted"], (f.name, r)
    return res


@pytest.mark.parametrize("k", [4, 10, 18])
def test_count_totals_match_oracle(ctx, k):
    cnfs = _formulas(211, ((16, 2.0), (20, 3.0), (24, 4.26), (28, 4.26), (30, 3.5), (32, 4.26), (36, 2.5),
                           (40, 4.26)))
    _count_totals(ctx, cnfs, k)


def test_count_totals_small_steps(ctx):
    """split_batch = 3: a step pops at most three nodes, so the stack holds
    many levels at once and every query's tree is interleaved with the
    others'."""
    cnfs = _formulas(212, ((20, 4.26), (26, 4.26), (30, 3.0), (34, 4.26)))
    _count_totals(ctx, cnfs, 8, split_batch=3)


def test_count_pigeonhole_and_degenerate(ctx):
    from workloads.cnf import CNF
    cnfs = [w.pigeonhole(4, 4), w.pigeonhole(5, 4), w.pigeonhole(4, 3), w.pigeonhole(3, 3)]
    # a formula whose root fixes every variable, and one with a single clause
    cnfs.append(CNF(3, np.array([0, 1, 2, 3], np.uint64), np.array([1, -2, 3], np.int32), name="units"))
    cnfs.append(CNF(5, np.array([0, 2], np.uint64), np.array([1, -5], np.int32), name="one_clause"))
    for k in (1, 6, 16):
        _count_totals(ctx, cnfs, k)


@pytest.mark.parametrize("k", [12, 20])
def test_decide_random_3sat_matches_oracle(ctx, k):
    cnfs = _formulas(213, [(n, 4.26) for n in (50, 60, 70, 80) for _ in range(12)])
    raw = _raw(ctx, cnfs)
    res = ctx.decide(raw, k=k, device_split=True, max_cubes=1 << 22)
    host = ctx.decide(raw, k=k, max_cubes=1 << 22)
    for qi, f in enumerate(cnfs):
        want = cnf_ref.solve(f)[0]
        r = res.result(qi)
        assert r["verdict"] == want, (f.name, r, want)
        assert host.result(qi)["verdict"] == want, (f.name, host.result(qi))
        if want == "SAT":
            assert r["witness_checked"]
            model = res.model(qi, f.n_vars)
            assert cnf_ref.check_model(f, model), f.name


def test_decide_pigeonhole(ctx):
    cnfs = [w.pigeonhole(5, 4), w.pigeonhole(6, 5), w.pigeonhole(5, 5), w.pigeonhole(7, 6)]
    res = ctx.decide(_raw(ctx, cnfs), k=10, device_split=True, max_cubes=1 << 22)
    assert res.verdicts() == ["UNSAT", "UNSAT", "SAT", "UNSAT"]


@pytest.mark.parametrize("scorer", ["static", "word"])
def test_decide_access_batches(ctx, scorer):
    """Bit-blasted access queries: every verdict is the label or UNKNOWN
    (the device tree has no word-level bounds, so a budget can run out where
    the host split prunes), every SAT witness passes the exact integer
    query, and the queries the root stage leaves open are mostly decided."""
    gens = w.batch_1d() + w.batch_2d(seed=33, n=96, wmax=14)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=20, device_split=True, scorer=scorer, max_cubes=20000)
    unknown = 0
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] in (g.label, "UNKNOWN"), (g.query.name, r)
        unknown += r["verdict"] == "UNKNOWN"
        if r["verdict"] == "UNKNOWN":
            assert r["how"] == "budget", r
        if r["verdict"] == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars)), g.query.name
    assert unknown <= len(gens) // 8, unknown


def test_budget_leaves_unknown(ctx):
    cnfs = [w.pigeonhole(8, 7)]
    res = ctx.decide(_raw(ctx, cnfs), k=4, device_split=True, max_cubes=50)
    r = res.result(0)
    assert r["verdict"] == "UNKNOWN" and r["how"] == "budget", r
    assert r["cubes_total"] >= 50


def _dense_planted(n, m, rng, name):
    """m random clauses of 3..6 distinct variables over n variables, each
    keeping a literal that a hidden assignment makes true: satisfiable,
    with few models, and more clauses than the wide-split threshold."""
    from workloads.cnf import CNF
    hidden = rng.integers(0, 2, size=n + 1).astype(bool)
    offs, lits = [0], []
    for _ in range(m):
        k = int(rng.integers(3, 7))
        vs = rng.choice(n, size=k, replace=False) + 1
        sg = rng.integers(0, 2, size=k).astype(bool)
        if not any(hidden[v] == s for v, s in zip(vs, sg)):
            j = int(rng.integers(0, k))
            sg[j] = hidden[vs[j]]
        lits.extend(int(v) if s else -int(v) for v, s in zip(vs, sg))
        offs.append(len(lits))
    return CNF(n, np.array(offs, np.uint64), np.array(lits, np.int32), name=name)


@pytest.mark.parametrize("k", [6, 14])
def test_wide_count_totals_match_oracle(ctx, k):
    """Queries of 16,384 clauses or more split wide: a node's slots are its
    unassigned variables, one node per query and step.  The leaves still
    add up to the oracle's exact model count; one small query rides along in
    the same batch."""
    rng = np.random.Generator(np.random.PCG64(214 + k))
    cnfs = [_dense_planted(26, 17000 + 1000 * i, rng, f"wide{i}") for i in range(3)]
    cnfs += _formulas(215, ((22, 3.0),))
    assert max(f.n_clauses for f in cnfs) >= 16384
    _count_totals(ctx, cnfs, k)


def test_wide_decide_access_batch(ctx):
    """Full-width 2-D accesses (their CNFs reach 80,000 clauses): every
    verdict is the label or UNKNOWN, every SAT witness passes the exact
    integer query, and the host split agrees where both decide."""
    gens = w.batch_2d(seed=35, n=192)
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, device_split=True, scorer="word", max_cubes=20000)
    host = ctx.decide(cnf, k=30, scorer="word", max_cubes=20000)
    unknown = 0
    for i, g in enumerate(gens):
        r, h = res.result(i), host.result(i)
        assert r["verdict"] in (g.label, "UNKNOWN"), (g.query.name, r)
        assert "UNKNOWN" in (r["verdict"], h["verdict"]) or r["verdict"] == h["verdict"], (g.query.name, r, h)
        unknown += r["verdict"] == "UNKNOWN"
        if r["verdict"] == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars)), g.query.name
    assert unknown <= len(gens) // 16, unknown
