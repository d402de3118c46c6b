"""The allocation-free decide entry point against scuba_decide: two calls
in a row on the library's device scratch, the second with a smaller batch,
each compared query by query with the workspace form (verdicts, how they
were reached, leaves sent and refuted, cubes, and the witness itself, which both forms
pick as the smallest (cube, assignment) key)."""
import numpy as np
import pytest

from oracle import query_ref
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _compare(ctx, gens, opts):
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    ref = ctx.decide(cnf, **opts)
    got = ctx.decide_noalloc(cnf, **opts)
    for i, g in enumerate(gens):
        a, b = ref.result(i), got.result(i)
        # (blocks evaluated before a query's early exit depend on timing)
        for key in ("verdict", "how", "leaves_sent", "leaves_refuted", "cubes_total", "cubes_refuted"):
            assert a[key] == b[key], (i, key, a, b)
        assert b["verdict"] in (g.label, "UNKNOWN"), (i, b)
        if b["verdict"] == "SAT":
            assert b["witness_checked"]
            wa = ref.witness(i, g.query.n_vars)
            wb = got.witness(i, g.query.n_vars)
            assert list(wa) == list(wb), (i, wa, wb)
            assert query_ref.int_eval(g.query, wb)
    return got


def test_noalloc_two_calls(ctx):
    # first call: 96 mixed 1-D queries, two leaves per query per round
    big = w.batch_1d(seed=31, n=96)
    _compare(ctx, big, dict(k=30, leaves_per_round=2, chunk_log2=8))
    # second call: a smaller batch of other queries; the scratch still holds
    # the first call's data
    small = w.batch_1d(seed=32, n=24)
    _compare(ctx, small, dict(k=24, leaves_per_round=1, chunk_log2=10))
    # and 2-D queries of several widths, static and word orderings
    two = w.batch_2d(seed=33, n=40, wmax=14)
    _compare(ctx, two, dict(k=20, max_cubes=20000))
    _compare(ctx, two[:12], dict(k=20, max_cubes=20000, scorer="word"))
