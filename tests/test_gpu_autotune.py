"""The autotuner: its choice lies in the sweep, a second call is served
from the cache, and verdicts do not depend on the tuning point (every
coordinate value of the sweep gives the generators' labels)."""
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


@pytest.fixture(scope="module")
def batch(ctx):
    gens = w.batch_2d(n=512) + w.batch_1d()[:128]
    return gens, ctx.bitblast([g.query.arrays()[:2] for g in gens])


def test_autotune_choice_and_cache(ctx, batch):
    gens, cnf = batch
    opts, rep = ctx.autotune(cnf, sample=48, reps=1, scorer="word")
    assert rep["points"] >= 5 and not rep["cached"]
    assert rep["best_ms"] <= rep["default_ms"]
    assert opts["k"] in (16, 20, 24, 28, 30)
    assert opts["chunk_log2"] in (4, 6, 8, 10, 12)
    assert opts["leaves_per_round"] in (1, 2, 4, 8, 16)
    assert opts["max_residual"] in (1024, 2048, 4096, 8192)
    assert opts["scorer"] == "word"
    again, rep2 = ctx.autotune(cnf, sample=48, reps=1, scorer="word")
    assert rep2["cached"] and again == opts
    res = ctx.decide(cnf, **opts)
    assert res.verdicts() == [g.label for g in gens]


@pytest.mark.parametrize("point", [
    dict(k=16), dict(k=24), dict(k=30),
    dict(chunk_log2=4), dict(chunk_log2=12),
    dict(leaves_per_round=1), dict(leaves_per_round=16),
    dict(grid=512), dict(grid=4096),
    dict(max_residual=1024), dict(max_residual=8192),
    dict(k=20, chunk_log2=6, leaves_per_round=2, graph=True),
])
def test_verdicts_do_not_depend_on_the_point(ctx, batch, point):
    gens, cnf = batch
    res = ctx.decide(cnf, scorer="word", max_cubes=20000, **point)
    assert res.verdicts() == [g.label for g in gens], point
