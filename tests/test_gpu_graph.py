"""Rounds captured as HIP graphs: every replay gives the eager path's
results (verdicts, counters, witnesses, per-leaf counts), with eager work
and synchronisations between the replays; a batch solved again replays
without capturing."""
import numpy as np
import pytest

from oracle import cnf_ref
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _summary(res, n, nvars):
    """What DECIDE fixes: verdicts, witnesses (the smallest key), cubes and
    leaves per query and rounds.  Blocks evaluated are left out: in DECIDE
    mode other waves stop when they see the witness key, so the count
    depends on scheduling."""
    out = []
    for i in range(n):
        r = res.result(i)
        wit = res.witness(i, nvars[i]) if r["verdict"] == "SAT" else None
        out.append((r["verdict"], r["cubes_total"], r["leaves_sent"], r["leaves_refuted"],
                    r["rounds"], tuple(wit) if wit else None))
    return out


def test_decide_graph_replays_match_eager(ctx):
    import torch
    gens = w.batch_1d()
    nvars = [g.query.n_vars for g in gens]
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    eager = _summary(ctx.decide(cnf, k=30), len(gens), nvars)
    captures = []
    for rep in range(4):
        res = ctx.decide(cnf, k=30, graph=True)
        tm = res.timing()
        assert tm["graph_launches"] > 0 and tm["up_launches"] == 0
        captures.append(tm["graph_captures"])
        assert _summary(res, len(gens), nvars) == eager, rep
        # eager work of the program between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        assert float((x * 2).sum()) == float(x.sum()) * 2
        torch.cuda.synchronize()
        assert _summary(ctx.decide(cnf, k=30), len(gens), nvars) == eager
    assert captures[0] > 0 and all(c == 0 for c in captures[1:]), captures


def test_count_graph_replays_match_eager(ctx):
    rng = np.random.Generator(np.random.PCG64(301))
    cnfs = [w.random_ksat(n, int(round(4.0 * n)), 3, rng) for n in (20, 28, 36)]
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    cubes = ctx.split(raw, k=10)
    eager = ctx.solve(raw, cubes, mode=1)
    for rep in range(3):
        res = ctx.solve(raw, cubes, mode=1, graph=True)
        total = 0
        for qi, f in enumerate(cnfs):
            n = len(cubes.view(qi)["kind"])
            for c in range(n):
                assert res.leaf(qi, c) == eager.leaf(qi, c), (rep, qi, c)
            total += sum(res.leaf(qi, c)["count"] << max(res.leaf(qi, c)["m"], 0)
                         for c in range(n) if not res.leaf(qi, c)["refuted"])
        if rep == 0:
            assert total == sum(cnf_ref.count(f) for f in cnfs)
        ctx.solve(raw, cubes, mode=1)   # eager in between


def test_graph_key_covers_cube_grouping(ctx):
    """Two solves whose rounds have the same sizes (queries, cubes, literals,
    work items) but group their cubes differently (300 cubes split 100/200,
    then 102/198: 75 against 76 workgroup groups of up to four cubes of one
    query) must not share a captured graph: each replay equals the eager
    results of its own cube list."""
    rng = np.random.Generator(np.random.PCG64(302))
    f = w.random_ksat(24, 80, 3, rng)
    raw = ctx.cnf_from_arrays(*w.concat([f, f]))
    for split in ((100, 200), (102, 198), (100, 200)):
        cubes = ctx.cubes_from_arrays(raw, [[[1]] * split[0], [[-1]] * split[1]])
        eager = ctx.solve(raw, cubes, mode=1)
        res = ctx.solve(raw, cubes, mode=1, graph=True)
        for qi in range(2):
            for c in range(split[qi]):
                assert res.leaf(qi, c) == eager.leaf(qi, c), (split, qi, c)
        ref = cnf_ref.leaf(f, [1])
        assert eager.leaf(0, 0)["refuted"] == ref["refuted"]
        if not ref["refuted"]:
            assert (eager.leaf(0, 0)["f"], eager.leaf(0, 0)["count"]) == (ref["f"], ref["count"])
