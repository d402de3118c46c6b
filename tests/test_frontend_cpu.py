"""The query front-end (host and kernel analysis, paper Sec. 5.1 Fig. 9a/9b)
against the program interpreter, on the CPU: every query it emits, decided
by brute force over the query's own inputs, must give the interpreter's
verdict for that (launch, access, bound), and every satisfying assignment
must replay as an out-of-bounds access in the interpreter."""
import pytest

from oracle import program_ref as pr
from oracle import query_ref as qr
from paper_2601_21552_amd import frontend as fe
import workloads.program as P


def _check(prog):
    truth = pr.brute_force(prog, lower=True)
    aqs = fe.analyse(prog, lower=True)
    assert [a.key for a in aqs] == pr.keys(prog, lower=True)
    for a in aqs:
        verdict, count, first = qr.int_bruteforce(a.query)
        assert (verdict == "SAT") == truth[a.key][0], (prog.name, a.key, a.access)
        if verdict == "SAT":
            vals = dict(zip(a.query.var_names, first))
            assert pr.witness_goes_out(prog, a.key, vals), (prog.name, a.key, vals)
    return aqs, truth


@pytest.mark.parametrize("name", list(P.EXAMPLES))
def test_examples(name):
    prog = P.parse(P.EXAMPLES[name], name)
    aqs, truth = _check(prog)
    assert any(truth[a.key][0] for a in aqs)            # every example has a bug
    assert not all(truth[a.key][0] for a in aqs)        # and safe accesses


def test_random_programs():
    progs = P.random_programs(seed=11, n=24)
    n_sat = n = 0
    for prog in progs:
        aqs, truth = _check(prog)
        n += len(aqs)
        n_sat += sum(truth[a.key][0] for a in aqs)
    assert 0 < n_sat < n


def test_programs_with_host_branches():
    # launches under host branches: their conditions join the queries
    n_sat = n = 0
    for prog in P.uaf_examples() + P.random_uaf_programs(seed=24, n=24):
        aqs, truth = _check(prog)
        n += len(aqs)
        n_sat += sum(truth[a.key][0] for a in aqs)
    assert 0 < n_sat < n


def test_query_shape():
    prog = P.parse(P.EXAMPLES["guarded_grid"], "guarded_grid")
    aqs = fe.analyse(prog)
    assert [a.key for a in aqs] == [(0, "scale", 0, "upper"), (0, "scale", 1, "upper"),
                                    (1, "scale_le", 0, "upper")]
    assert [a.region for a in aqs] == ["global"] * 3
    q = aqs[2].query
    # the ids of the launch (8 blocks of 32 at most), then the input met in
    # the grid size
    assert q.var_names == ["threadIdx.x", "blockIdx.x", "n"]
    assert q.var_widths == [5, 3, 8]
    # kind 1 on x (two roots), the guard, the OOB test
    assert len(q.roots) == 4
    regions = {a.region for a in fe.analyse(P.parse(P.EXAMPLES["shm_partitions"]))}
    assert regions == {"global", "partition"}


def test_asserts_after_a_launch_do_not_constrain_it():
    prog = P.parse("""
        input n : 4
        malloc A = n
        launch k grid(1) block(16) args(A)
        assert n >= 16
        kernel k(a) { load a[threadIdx.x] }
    """, "late_assert")
    aqs, truth = _check(prog)
    assert truth[(0, "k", 0, "upper")][0]


def test_launches_under_host_branches():
    # the launch of the small-n branch can run past A; the other cannot
    prog = P.parse("""
        input n : 4
        malloc A = n
        if (n < 4) { launch k grid(1) block(4) args(A) }
        else { launch k grid(1) block(4) args(A) }
        kernel k(a) { load a[threadIdx.x] }
    """, "host_branches")
    aqs, truth = _check(prog)
    assert truth[(0, "k", 0, "upper")][0]
    assert not truth[(1, "k", 0, "upper")][0]


@pytest.mark.parametrize("text,match", [
    ("input n : 4\nlet m = k + 1", "before its definition"),
    ("input n : 4\nlet n = 3", "defined twice"),
    ("input n : 4\nassert n", "bool expected"),
    ("input n : 4\nlet m = n / n", "literal on the right"),
    ("input n : 4\nlet m = n % 0", "literal on the right"),
    ("input n : 0", "1..64 bits"),
    ("kernel k(a) { load a[0] shared s[4] }", "precede the accesses"),
    ("kernel k(a) { if (a < 1) { shared s[4] } }", "top level"),
    ("kernel k(a) { partition p = a + 1 }", "not a dynamic shared base"),
    ("kernel k(a) { load b[0] }", "unknown b"),
    ("input n : 4\nlaunch k grid(1) block(1) args(n, n)\nkernel k(a) { }", "takes 1 arguments"),
    ("input n : 4\nlaunch q grid(1) block(1) args()", "unknown kernel"),
    ("kernel k(a) { let t = threadIdx.w }", "unknown builtin"),
    ("input n : 4\nfree n", "not a malloc'd buffer"),
    ("input n : 4\nif (n < 2) { let m = 3 }", "inside a host branch"),
    ("kernel k(a) { shared s[2] free s }", "not a parameter"),
])
def test_parse_errors(text, match):
    with pytest.raises(P.ParseError, match=match):
        P.parse(text)


def test_frontend_rejections():
    # a pointer used as a value, and a division that may see a negative value
    bad_ptr = P.parse("""
        input n : 4
        malloc A = n
        launch k grid(1) block(4) args(A)
        kernel k(a) { load a[a] }
    """)
    with pytest.raises(fe.FrontendError, match="pointer"):
        fe.analyse(bad_ptr)
    bad_div = P.parse("""
        input n : 4
        malloc A = n
        launch k grid(1) block(4) args(A, n)
        kernel k(a, len) { load a[(threadIdx.x - 2) / 2] }
    """)
    with pytest.raises(fe.FrontendError, match="negative"):
        fe.analyse(bad_div)
    wide = P.parse("""
        input n : 40
        malloc A = n
        launch k grid(n * n) block(1) args(A)
        kernel k(a) { load a[blockIdx.x] }
    """)
    with pytest.raises(fe.FrontendError, match="64 bits"):
        fe.analyse(wide)
