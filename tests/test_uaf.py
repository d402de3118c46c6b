"""Use-after-free detection by live sets (paper Sec. 4.3, Sec. 5.3) against
the program interpreter, which tracks which buffers are really live in every
run.  The analysis is path-insensitive, so it must report every use after
free that some run performs (sound), and exactly those when every branch
tests an input of its own (all paths feasible)."""
import re

from oracle import program_ref as pr
from paper_2601_21552_amd import uaf
import workloads.program as P


def _prog(name):
    return P.parse(P.UAF_EXAMPLES[name], name)


def test_free_then_launch():
    # launch 1 passes A after a free on one path; launch 2 passes both after
    # B's unconditional free
    want = {("uaf", "launch", 1, "k", 0), ("uaf", "launch", 2, "k", 0),
            ("uaf", "launch", 2, "k", 1)}
    p = _prog("free_then_launch")
    assert uaf.analyse(p) == want
    assert pr.uaf_brute_force(p) == want


def test_device_free():
    # accesses: 0 load p[0], 1 store s[t], 2 load q[j] (after the previous
    # iteration's free), 3 load p[1] (after the branch's free)
    want = {("uaf", "access", "k", 2), ("uaf", "access", "k", 3)}
    p = _prog("device_free")
    assert uaf.analyse(p) == want
    assert pr.uaf_brute_force(p) == want


def test_correlated_branches_are_a_false_report():
    p = _prog("correlated_branches")
    assert uaf.analyse(p) == {("uaf", "launch", 0, "k", 0)}
    assert pr.uaf_brute_force(p) == set()


def test_random_programs_exact():
    n_reports = 0
    for p in P.random_uaf_programs(seed=21, n=64):
        got, truth = uaf.analyse(p), pr.uaf_brute_force(p)
        assert got == truth, (p.name, sorted(got ^ truth))
        n_reports += len(truth)
    assert n_reports > 100


def test_random_programs_sound_with_shared_conditions():
    # every host branch tests the same input: some reported uses can no
    # longer happen, but every use that happens is reported
    extra = 0
    for p in P.random_uaf_programs(seed=22, n=64):
        q = P.parse(re.sub(r"\(c\d+ ==", "(c0 ==", p.text), p.name + "_shared")
        got, truth = uaf.analyse(q), pr.uaf_brute_force(q)
        assert truth <= got, (q.name, sorted(truth - got))
        extra += len(got - truth)
    assert extra > 0


def test_programs_without_frees_are_clean():
    for p in P.examples() + P.random_programs(seed=11, n=24):
        assert uaf.analyse(p) == set()
        assert pr.uaf_brute_force(p) == set()
