"""Edge cases of DECIDE through the C ABI: an empty batch, a batch that the
root stage decides entirely (nothing uploaded, no kernel launched), the same
CNF decided twice (the upload's staging reused), root-decided queries mixed
with device queries, and options outside the documented limits."""
import pytest

from oracle import query_ref
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _summary(res, gens):
    out = []
    for i, g in enumerate(gens):
        r = res.result(i)
        wit = tuple(res.witness(i, g.query.n_vars)) if r["verdict"] == "SAT" else None
        out.append((r["verdict"], r["how"], r["cubes_total"], r["leaves_sent"], wit))
    return out


def test_empty_batch(ctx):
    cnf = ctx.bitblast([])
    res = ctx.decide(cnf, k=30)
    assert res.verdicts() == []
    tm = res.timing()
    assert tm["up_launches"] == 0 and tm["leaf_launches"] == 0


def test_batch_decided_at_the_root(ctx):
    gens = [g for g in w.batch_1d() if g.kind.startswith("guarded")]
    assert gens
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label == "UNSAT"
        assert r["how"] == "root" and r["leaves_sent"] == 0
    tm = res.timing()
    assert tm["up_launches"] == 0 and tm["leaf_launches"] == 0


def test_mixed_batch_and_repeat(ctx):
    # root-decided queries interleaved with device ones, decided twice on one
    # CNF handle: the second call must give the first call's results
    gens = w.batch_1d()[::3] + [w.single_access("lt"), w.single_access("none")]
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    first = ctx.decide(cnf, k=30, leaves_per_round=1, chunk_log2=12)
    again = ctx.decide(cnf, k=30, leaves_per_round=1, chunk_log2=12)
    assert _summary(first, gens) == _summary(again, gens)
    for i, g in enumerate(gens):
        r = first.result(i)
        assert r["verdict"] == g.label, g.query.name
        if g.label == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, first.witness(i, g.query.n_vars))


def test_options_beyond_the_limits_are_rejected(ctx):
    from paper_2601_21552_amd._lib import ScubaError
    cnf = ctx.bitblast([w.single_access("none").query.arrays()[:2]])
    with pytest.raises(ScubaError):
        ctx.decide(cnf, k=39)
