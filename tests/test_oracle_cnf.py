"""Pins of the CPU DPLL oracle against facts it does not compute itself:
brute force over every assignment of tiny formulas, the pigeonhole
principle's textbook closed forms, and a replay check of the propagation
fixpoint.  CPU only."""
import math

import numpy as np
import pytest

from oracle import cnf_ref
from workloads import CNF, pigeonhole, random_ksat
import workloads as w


def _rand_cnfs(seed, count, nmax=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.integers(3, nmax + 1))
        k = int(rng.integers(1, 4)) if n >= 3 else 1
        ratio = float(rng.choice([1.0, 2.5, 4.3, 6.0]))
        m = max(1, int(ratio * n))
        out.append(random_ksat(n, m, min(k + 1, 3, n), rng))
    return out


def test_decide_matches_brute_force():
    for cnf in _rand_cnfs(11, 120):
        cnt, _ = cnf_ref.brute_force(cnf)
        verdict, model, _ = cnf_ref.solve(cnf)
        assert verdict == ("SAT" if cnt else "UNSAT"), cnf.name
        if model is not None:
            assert cnf_ref.check_model(cnf, model)


def test_count_matches_brute_force():
    for cnf in _rand_cnfs(12, 120):
        cnt, _ = cnf_ref.brute_force(cnf)
        assert cnf_ref.count(cnf) == cnt


def test_free_variables_double_the_count():
    # a variable in no clause contributes a factor two
    cnf = CNF.from_clauses(5, [[1, 2], [-1, 3]])
    assert cnf_ref.count(cnf) == cnf_ref.brute_force(cnf)[0] == 4 * 4


def test_degenerate_formulas():
    empty = CNF.from_clauses(3, [])
    assert cnf_ref.solve(empty)[0] == "SAT"
    assert cnf_ref.count(empty) == 8
    with_empty_clause = CNF.from_clauses(2, [[1], []])
    assert cnf_ref.solve(with_empty_clause)[0] == "UNSAT"
    assert cnf_ref.count(with_empty_clause) == 0
    assert cnf_ref.leaf(with_empty_clause)["refuted"]


@pytest.mark.parametrize("h", [1, 2, 3, 4, 5])
def test_pigeonhole_unsat(h):
    assert cnf_ref.solve(pigeonhole(h + 1, h))[0] == "UNSAT"


@pytest.mark.parametrize("h", [1, 2, 3, 4, 5, 6])
def test_pigeonhole_bijections(h):
    # h pigeons in h holes: the models are exactly the h! bijections
    assert cnf_ref.count(pigeonhole(h, h)) == math.factorial(h)


def _replays_by_unit_steps(cnf, cube, assign):
    """The fixpoint must be reachable from the cube by unit steps alone and
    leave no unit or empty clause behind."""
    cur = {abs(l): int(l > 0) for l in cube}
    clauses = cnf.clauses()
    grew = True
    while grew:
        grew = False
        for cl in clauses:
            if any(cur.get(abs(l)) == int(l > 0) for l in cl):
                continue
            open_ = [l for l in cl if abs(l) not in cur]
            if len(open_) == 1:
                v, val = abs(open_[0]), int(open_[0] > 0)
                if assign[v] != val:
                    return False
                cur[v] = val
                grew = True
    fix = {v: int(assign[v]) for v in range(1, cnf.n_vars + 1) if assign[v] >= 0}
    if fix != cur:
        return False
    for cl in clauses:
        if any(fix.get(abs(l)) == int(l > 0) for l in cl):
            continue
        if sum(abs(l) not in fix for l in cl) < 2:
            return False
    return True


def _random_cube(rng, n, size):
    vs = rng.choice(n, size=size, replace=False) + 1
    return [int(v) if rng.integers(2) else -int(v) for v in vs]


def test_leaf_against_brute_force():
    rng = np.random.Generator(np.random.PCG64(13))
    checked = 0
    for cnf in _rand_cnfs(14, 80, nmax=12):
        cnt_all, models = cnf_ref.brute_force(cnf)
        for _ in range(4):
            cube = _random_cube(rng, cnf.n_vars, int(rng.integers(0, 4)))
            lf = cnf_ref.leaf(cnf, cube)
            conflict, assign = cnf_ref.up(cnf, cube)
            # models consistent with the cube
            mask = np.ones(len(models), dtype=bool)
            for l in cube:
                bit = (models >> (abs(l) - 1)) & 1
                mask &= (bit == 1) if l > 0 else (bit == 0)
            sub = models[mask]
            if lf["refuted"]:
                assert conflict and len(sub) == 0
                continue
            assert not conflict
            assert _replays_by_unit_steps(cnf, cube, assign)
            # every propagated value is forced in every model of F and cube
            for v in range(1, cnf.n_vars + 1):
                if assign[v] >= 0 and len(sub):
                    assert np.all(((sub >> (v - 1)) & 1) == assign[v])
            # active set: unassigned variables of unsatisfied clauses
            act = set()
            for cl in cnf.clauses():
                if any(assign[abs(l)] == int(l > 0) for l in cl):
                    continue
                act |= {abs(l) for l in cl if assign[abs(l)] < 0}
            assert lf["slots"] == sorted(act)
            free = [v for v in range(1, cnf.n_vars + 1) if assign[v] < 0]
            assert lf["f"] == len(act) and lf["m"] == len(free) - len(act)
            assert lf["count"] * 2 ** lf["m"] == len(sub)
            # smallest satisfying slot index, by enumeration of 2**f
            best = -1
            fixed = sum(1 << (v - 1) for v in range(1, cnf.n_vars + 1)
                        if assign[v] == 1)
            subset = set(int(x) for x in sub)
            for a in range(1 << lf["f"]):
                word = fixed
                for j, v in enumerate(lf["slots"]):
                    if (a >> j) & 1:
                        word |= 1 << (v - 1)
                if word in subset:
                    best = a
                    break
            assert lf["first"] == best
            checked += 1
    assert checked > 100


def test_leaf_counts_partition_the_models():
    """Sum over a complete, disjoint cube set of count * 2**m is #SAT."""
    rng = np.random.Generator(np.random.PCG64(15))
    for cnf in _rand_cnfs(16, 30, nmax=12):
        total, _ = cnf_ref.brute_force(cnf)
        vs = [int(v) for v in rng.choice(cnf.n_vars, size=3, replace=False) + 1]
        acc = 0
        for bits in range(8):
            cube = [v if (bits >> i) & 1 else -v for i, v in enumerate(vs)]
            lf = cnf_ref.leaf(cnf, cube)
            if not lf["refuted"]:
                acc += lf["count"] * 2 ** lf["m"]
        assert acc == total


def test_threshold_3sat_is_decided():
    rng = np.random.Generator(np.random.PCG64(17))
    for n in (20, 40):
        for _ in range(5):
            cnf = random_ksat(n, int(round(4.26 * n)), 3, rng)
            v, model, _ = cnf_ref.solve(cnf)
            assert v in ("SAT", "UNSAT")
            if v == "SAT":
                assert cnf_ref.check_model(cnf, model)
            if n == 20:
                assert (v == "SAT") == (cnf_ref.brute_force(cnf)[0] > 0)


def test_random_ksat_batch_model():
    """Batch generator of the random k-SAT model: k distinct variables per
    clause in range, signs and variables close to uniform."""
    rng = np.random.Generator(np.random.PCG64(44))
    fs = w.random_ksat_batch(50, 213, 3, 40, rng)
    assert len(fs) == 40 and all(f.n_clauses == 213 and f.n_vars == 50 for f in fs)
    lits = np.stack([f.lits.reshape(-1, 3) for f in fs])
    v = np.abs(lits)
    assert v.min() >= 1 and v.max() <= 50
    s = np.sort(v, axis=2)
    assert (s[:, :, 1:] != s[:, :, :-1]).all()
    cnt = np.bincount(v.ravel(), minlength=51)[1:]
    expect = v.size / 50
    chi2 = float(((cnt - expect) ** 2 / expect).sum())
    assert chi2 < 100, chi2          # 49 degrees of freedom
    assert abs((lits > 0).mean() - 0.5) < 0.02
