"""The learned branching scorer inside the solver (GPU).

* Any network, trained or not, only reorders decisions: learned cube sets
  stay complete and disjoint (their counts add up to the oracle's model
  count) and decide() gives the oracle's verdicts with verified witnesses.
* Trained on the splitter's own traces (forward, backward and Adam in the
  library's kernels), the scorer shrinks held-out random 3-SAT trees
  against the static most-occurrences ordering.
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


@pytest.fixture(scope="module")
def untrained(ctx):
    from paper_2601_21552_amd import api, train
    return api.Mlp(ctx, train._he_init(np.random.Generator(np.random.PCG64(9))))


def _sat_batch(n, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [w.random_3sat_threshold(n, rng) for _ in range(count)]


def test_learned_split_is_a_partition(ctx, untrained):
    cnfs = _sat_batch(30, 6, 201) + _sat_batch(40, 4, 202)
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    sc = untrained.scorer(candidates=12, rescore=1)
    for k in (6, 10):
        learned = ctx.split(raw, k=k, learned=sc)
        static = ctx.split(raw, k=k)
        differ = False
        out = ctx.solve(raw, learned, mode=1)
        for qi, f in enumerate(cnfs):
            v = learned.view(qi)
            assert v["complete"]
            differ |= v["cubes"] != static.view(qi)["cubes"]
            total = 0
            for c, cube in enumerate(v["cubes"]):
                lf = out.leaf(qi, c)
                if v["kind"][c] == 2:
                    assert lf["refuted"]
                    continue
                ref = cnf_ref.leaf(f, cube)
                assert lf["refuted"] == ref["refuted"], (qi, c)
                if not ref["refuted"]:
                    assert (lf["f"], lf["m"], lf["count"], lf["first"]) == \
                        (ref["f"], ref["m"], ref["count"], ref["first"]), (qi, c)
                    total += lf["count"] << lf["m"]
            assert total == cnf_ref.count(f), qi
        assert differ, "the learned ordering never departed from the static one"


def test_learned_decide_verdicts(ctx, untrained):
    sc = untrained.scorer(candidates=16, rescore=2)
    cnfs = _sat_batch(50, 24, 203)
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    res = ctx.decide(raw, k=12, learned=sc)
    for qi, f in enumerate(cnfs):
        want, _, _ = cnf_ref.solve(f)
        r = res.result(qi)
        assert r["verdict"] == want, qi
        if want == "SAT":
            assert cnf_ref.check_model(f, res.model(qi, f.n_vars))
    gens = w.batch_1d()[:96]
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    res = ctx.decide(cnf, k=30, learned=sc)
    for i, g in enumerate(gens):
        r = res.result(i)
        assert r["verdict"] == g.label, (g.query.name, r)
        if g.label == "SAT":
            assert r["witness_checked"]
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))


def test_trained_scorer_shrinks_trees(ctx):
    from paper_2601_21552_amd import train
    k = 12
    tr = [ctx.cnf_from_arrays(*w.concat(_sat_batch(60, 48, 1000))),
          ctx.cnf_from_arrays(*w.concat(_sat_batch(80, 24, 1001)))]
    f, lab, nodes = train.collect(ctx, tr, k=k, candidates=16, depth=40)
    assert len(lab) > 10000
    mlp, hist = train.train(ctx, f, train.node_targets(lab, nodes), epochs=4, seed=1)
    assert hist[-1] < hist[0]
    held = _sat_batch(80, 24, 2080)
    raw = ctx.cnf_from_arrays(*w.concat(held))
    sc = mlp.scorer(candidates=16, rescore=1)

    def size(cubes):
        tot = leaves = 0
        for qi in range(len(held)):
            kind = cubes.view(qi)["kind"]
            tot += len(kind)
            leaves += int((kind == 0).sum())
        return tot, leaves

    st = size(ctx.split(raw, k=k))
    le = size(ctx.split(raw, k=k, learned=sc))
    assert le[0] < 0.75 * st[0], (le, st)
    assert le[1] < 0.75 * st[1], (le, st)
    # the same verdicts either way
    a = ctx.decide(raw, k=k).verdicts()
    b = ctx.decide(raw, k=k, learned=sc).verdicts()
    assert a == b
