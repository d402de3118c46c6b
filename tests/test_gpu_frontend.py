"""Programs through the whole path: the front-end's queries (paper Sec. 5.1
Fig. 9a/9b, Sec. 5.2) bit-blasted and decided on the GPU through the C ABI,
against the concrete interpreter that runs every input, block, thread and
loop iteration of the program.  Verdicts must agree for every (launch,
access, bound); every SAT witness must be checked by the library and must
replay as an out-of-bounds access in the interpreter."""
import pytest

from oracle import program_ref as pr
from paper_2601_21552_amd import frontend as fe
import workloads.program as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _decide(ctx, progs, **opts):
    aqs, truth = [], {}
    for p in progs:
        truth[p.name] = pr.brute_force(p, lower=True)
        aqs += [(p, a) for a in fe.analyse(p, lower=True)]
    print(f"{len(progs)} programs, {len(aqs)} queries", flush=True)
    cnf = ctx.bitblast([a.query.arrays()[:2] for _, a in aqs])
    res = ctx.decide(cnf, **opts)
    n_sat = 0
    for i, (p, a) in enumerate(aqs):
        r = res.result(i)
        want = "SAT" if truth[p.name][a.key][0] else "UNSAT"
        assert r["verdict"] == want, (p.name, a.key, a.access, r)
        if want == "SAT":
            n_sat += 1
            assert r["witness_checked"]
            vals = dict(zip(a.query.var_names, res.witness(i, a.query.n_vars)))
            assert pr.witness_goes_out(p, a.key, vals), (p.name, a.key, vals)
    return len(aqs), n_sat


def test_example_programs(ctx):
    n, n_sat = _decide(ctx, P.examples(), k=30)
    assert 0 < n_sat < n


def test_random_programs(ctx):
    n, n_sat = _decide(ctx, P.random_programs(seed=12, n=96), k=30,
                       leaves_per_round=1, chunk_log2=12)
    assert 0 < n_sat < n


def test_random_programs_small_leaves(ctx):
    # a small leaf bound sends the splitter below the root on most queries
    n, n_sat = _decide(ctx, P.random_programs(seed=13, n=48), k=4)
    assert 0 < n_sat < n


def test_programs_with_host_branches(ctx):
    progs = P.uaf_examples() + P.random_uaf_programs(seed=25, n=48)
    n, n_sat = _decide(ctx, progs, k=30)
    assert 0 < n_sat < n
