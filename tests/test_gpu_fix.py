"""The host-fixpoint check (fix_kernel) against the oracle on leaves with
thousands of unsatisfied clauses.

scuba_decide sends every leaf with the splitter's fixpoint, so its rounds
run fix_kernel: one pass over the clauses that confirms the fixpoint, marks
the active variables and lists the unsatisfied clauses for the residual
records.  These formulas keep most clauses open at their leaves, so:

* a wave lists more unsatisfied clauses than its LDS list holds, and the
  records come from the second pass over its clauses;
* clauses of up to ten literals take the path past the four literals that
  are loaded with the clause;
* CNFs from 4,000 to 24,000 clauses run with four-wave and eight-wave
  teams.

Verdicts equal the oracle's DPLL verdicts, and every SAT model satisfies
every clause, checked here again.
"""
import numpy as np
import pytest

from oracle import cnf_ref
from workloads.cnf import CNF
import workloads as w

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2601_21552_amd import api
    return api.Context(0)


def _dense(n, m, rng, planted, name):
    """m random clauses of 2..10 distinct variables over n variables (half of
    them of three); with `planted`, every clause keeps a literal that a
    hidden assignment makes true, so the formula is satisfiable."""
    hidden = rng.integers(0, 2, size=n + 1).astype(bool)
    offs, lits = [0], []
    for _ in range(m):
        k = 3 if rng.random() < 0.5 else int(rng.integers(2, 11))
        vs = rng.choice(n, size=k, replace=False) + 1
        sg = rng.integers(0, 2, size=k).astype(bool)
        if planted and not any(hidden[v] == s for v, s in zip(vs, sg)):
            j = int(rng.integers(0, k))
            sg[j] = hidden[vs[j]]
        lits.extend(int(v) if s else -int(v) for v, s in zip(vs, sg))
        offs.append(len(lits))
    return CNF(n, np.array(offs, np.uint64), np.array(lits, np.int32), name=name)


@pytest.mark.parametrize("m", [4000, 24000])
def test_dense_leaves_match_oracle(ctx, m):
    rng = np.random.Generator(np.random.PCG64(900 + m))
    cnfs = [_dense(18, m, rng, True, f"planted{i}") for i in range(3)]
    cnfs += [_dense(18, m, rng, False, f"open{i}") for i in range(2)]
    cnfs += [w.random_ksat(16, 8 * m // 10, 3, rng, name="ksat")]
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    res = ctx.decide(raw, k=14, max_residual=8192, max_cubes=1 << 16)
    assert res.timing()["fix_launches"] >= 1
    for qi, f in enumerate(cnfs):
        want = cnf_ref.solve(f)[0]
        r = res.result(qi)
        assert r["verdict"] == want, (f.name, r, want)
        if want == "SAT":
            assert r["witness_checked"]
            assert cnf_ref.check_model(f, res.model(qi, f.n_vars)), f.name


def test_small_cnfs_in_a_wide_launch(ctx):
    """One CNF of 20,000 clauses makes the launch give every cube an
    eight-wave team; the other CNFs have 1 to 70 clauses, so most of their
    team's waves get empty clause ranges and the rest end inside a 64-clause
    chunk.  Verdicts equal the oracle's."""
    rng = np.random.Generator(np.random.PCG64(4242))
    cnfs = [_dense(18, 20000, rng, True, "wide")]
    for m in (1, 2, 3, 17, 63, 64, 65, 70):
        cnfs.append(_dense(12, m, rng, m % 2 == 1, f"small{m}"))
    # every sign pattern of two variables (UNSAT with no unit clause: the
    # whole formula is one leaf), and a clashing pair of units
    cnfs.append(CNF(2, np.array([0, 2, 4, 6, 8], np.uint64),
                    np.array([1, 2, 1, -2, -1, 2, -1, -2], np.int32), name="all4"))
    cnfs.append(CNF(1, np.array([0, 1, 2], np.uint64), np.array([1, -1], np.int32), name="clash"))
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    res = ctx.decide(raw, k=14, max_residual=8192, max_cubes=1 << 16)
    assert res.timing()["fix_launches"] >= 1
    for qi, f in enumerate(cnfs):
        want = cnf_ref.solve(f)[0]
        r = res.result(qi)
        assert r["verdict"] == want, (f.name, r, want)
        if want == "SAT":
            assert r["witness_checked"]
            assert cnf_ref.check_model(f, res.model(qi, f.n_vars)), f.name
