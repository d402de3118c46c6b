"""Pins that hold the oracle's word-level side and the workloads' labels to
something other than themselves.  CPU only.

* The root check (the oracle's normal form, bound intersection and rational
  relaxation) is the same *method* as the library's root stage, so agreement
  between the two proves little.  Its soundness is pinned here against
  exhaustive integer search on random queries that use every operator,
  quotient and remainder atoms included, and root equalities that define
  one input from the others.
* The m-bit machine-integer evaluator is pinned by closed-form counts for
  wrapping multiplication, subtraction and shifts.
* Every generator family, in every variant, gets the verdict its label
  names from exhaustive search at small widths (2-4 bits per input): the
  full-width labels rest on constructions whose proofs do not depend on the
  width (an inequality chain for the correct guards, an explicit witness
  for the buggy ones), checked here by brute force, not by the root check.
* The guarded 1-D accesses are refuted by the oracle's own Tseitin encoding
  and plain DPLL, with the root check skipped, at every width the DPLL
  finishes in seconds.
"""
import numpy as np
import pytest

import workloads as w
from oracle import cnf_ref, query_ref
from tests.querygen import random_query
from workloads import Query, oob_1d, oob_2d, oob_lower_1d, partition_query


# ---------------------------------------------------------------- root check soundness

def _has_division_root(q):
    """True if some root reaches a quotient or remainder node."""
    from workloads.query import OP_UDIV, OP_UREM
    reach = set(q.roots)
    for i in range(len(q.nodes) - 1, -1, -1):
        if i in reach:
            op, a, b, _, _ = q.nodes[i]
            if op in (OP_UDIV, OP_UREM):
                return True
            reach.update((a, b))
    return False


def test_root_check_sound_with_quotients_and_remainders():
    """Queries over every operator, quotient and remainder by constants
    included: a root-check UNSAT is never contradicted by exhaustive search,
    and the division atoms' ranges are exercised in those refutations."""
    rng = np.random.Generator(np.random.PCG64(501))
    hits = div_hits = 0
    for i in range(500):
        q = random_query(rng, max_bits=10, n_ops=6,
                         ops=("add", "sub", "mul", "udiv", "urem", "udiv", "urem", "const"),
                         name=f"d{i}")
        if query_ref.root_check(q) == "UNSAT":
            hits += 1
            div_hits += _has_division_root(q)
            assert query_ref.int_bruteforce(q)[0] == "UNSAT", q.nodes
    assert hits >= 20 and div_hits >= 10, (hits, div_hits)


def _defined_query(rng, name):
    """Inputs x0..x(n-1), one of them defined by a root equality from the
    others (x_d = polynomial of the rest), plus comparisons over sums and
    products: the shape of an allocation size that is the sum of its parts."""
    q = Query(name)
    n = int(rng.integers(3, 5))
    xs = [q.var(f"x{i}", int(rng.integers(1, 3 if n == 4 else 4))) for i in range(n)]
    d = int(rng.integers(n))
    rest = [x for i, x in enumerate(xs) if i != d]
    expr = rest[0]
    for x in rest[1:]:
        expr = expr * x if rng.random() < 0.3 else expr + x
    if rng.random() < 0.5:
        expr = expr + int(rng.integers(0, 3))
    q.require(xs[d].eq(expr))
    terms = xs + [xs[a] * xs[b] for a, b in rng.integers(0, n, size=(2, 2))]
    for _ in range(int(rng.integers(1, 4))):
        a = terms[int(rng.integers(len(terms)))]
        b = terms[int(rng.integers(len(terms)))]
        c = int(rng.integers(0, 4))
        kind = int(rng.integers(4))
        q.require([a < b + c, a + c >= b, a <= b, (a - b) > c][kind])
    return q


def test_root_check_sound_with_defining_equalities():
    """A root equality that defines an input (substituted away by the root
    check) never turns a satisfiable query into an UNSAT verdict."""
    rng = np.random.Generator(np.random.PCG64(502))
    hits = 0
    for i in range(400):
        q = _defined_query(rng, f"e{i}")
        if query_ref.root_check(q) == "UNSAT":
            hits += 1
            assert query_ref.int_bruteforce(q)[0] == "UNSAT", q.nodes
    assert hits >= 20, hits


# ---------------------------------------------------------------- machine integers

@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_wrap_mul_zero_product_closed_form(m):
    """a*b = 0 mod 2^m.  For a = 0 every b; for a != 0 with 2-adic valuation
    v exactly the b that are multiples of 2^(m-v), i.e. 2^v of them.  There
    are 2^(m-1-v) values a of valuation v, so the count is
    2^m + sum_v 2^(m-1-v) 2^v = 2^m + m 2^(m-1).  With exact integers only
    a = 0 or b = 0: 2^(m+1) - 1 pairs."""
    q = Query("mul0")
    a, b = q.var("a", m), q.var("b", m)
    q.require((a * b).eq(0))
    assert query_ref.wrap_bruteforce(q, m)[1] == (1 << m) + m * (1 << (m - 1))
    assert query_ref.int_bruteforce(q)[1] == (1 << (m + 1)) - 1


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_wrap_sub_borrow_closed_form(m):
    """a - b > a (unsigned) holds exactly when b > a: then the difference
    wraps to a - b + 2^m > a; when b <= a it is a - b <= a.  That is
    2^m (2^m - 1) / 2 pairs; never with exact integers."""
    q = Query("sub")
    a, b = q.var("a", m), q.var("b", m)
    q.require((a - b) > a)
    assert query_ref.wrap_bruteforce(q, m)[1] == (1 << m) * ((1 << m) - 1) // 2
    assert query_ref.int_bruteforce(q)[0] == "UNSAT"


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_wrap_shl_and_mul_overflow_closed_forms(m):
    """(a << 1) < a holds exactly for a >= 2^(m-1) (2a - 2^m < a), i.e.
    2^(m-1) values; a*3 < a holds for the a with 3a mod 2^m < a: a in
    [2^m/3, 2^m/2) gives 3a - 2^m < a, a in [2^(m+1)/3, 2^m) gives
    3a - 2*2^m < a, counted here by the ceilings of those bounds."""
    q = Query("shl")
    a = q.var("a", m)
    q.require((a << 1) < a)
    assert query_ref.wrap_bruteforce(q, m)[1] == 1 << (m - 1)
    q3 = Query("mul3")
    a3 = q3.var("a", m)
    q3.require((a3 * 3) < a3)
    top = 1 << m
    ceil = lambda x, y: -(-x // y)                       # noqa: E731
    want = (ceil(top, 2) - ceil(top, 3)) + (top - ceil(2 * top, 3))
    assert query_ref.wrap_bruteforce(q3, m)[1] == want


# ---------------------------------------------------------------- generator families

def _bf(q):
    return query_ref.int_bruteforce(q)[0]


def _named(q, wit):
    return [wit[n] for n in q.var_names]


@pytest.mark.parametrize("width", [2, 3, 4])
def test_family_1d_labels_by_brute_force(width):
    """oob_1d in every variant the 1-D batches draw: the correct guard is
    UNSAT for every element size and header, the missing and off-by-one
    guards SAT (with the batch generator's witnesses)."""
    for s in (1, 2, 4, 8):
        for c in (0, 1, 7, 16):
            assert _bf(oob_1d(width, "lt", scale=s, header=c)) == "UNSAT", (width, s, c)
            for guard, wit in (("none", dict(N=0, blockDim=1, blockIdx=0, threadIdx=0)),
                               ("le", dict(N=1, blockDim=2, blockIdx=0, threadIdx=1))):
                q = oob_1d(width, guard, scale=s, header=c)
                assert _bf(q) == "SAT", (width, guard, s, c)
                assert query_ref.int_eval(q, _named(q, wit))


def test_family_2d_labels_by_brute_force():
    """oob_2d in all six kinds, with one, two and three multipliers, a
    separate row pitch, every element size and two headers: the label rule
    of the 2-D batch (correct -> UNSAT, each bug -> SAT with its witness)
    holds by exhaustive search wherever the inputs fit 22 bits."""
    checked = {"UNSAT": 0, "SAT": 0}
    for width in (2, 3):
        for guard in ("ok", "no_row", "no_col", "row_le", "col_le", "ld_free"):
            for mult in (1, 2, 3):
                for sep in ((False, True) if guard == "ok" else (False,)):
                    for s, c in ((1, 0), (2, 5), (4, 16), (8, 1)):
                        q = oob_2d(width, guard, mult, s, c, sep)
                        if q.input_bits > 22:
                            continue
                        want = "UNSAT" if guard == "ok" else "SAT"
                        assert _bf(q) == want, (width, guard, mult, sep, s, c)
                        if want == "SAT":
                            wit = w.generators._witness_2d(guard, mult, guard == "ld_free")
                            assert query_ref.int_eval(q, _named(q, wit))
                        checked[want] += 1
    assert checked["UNSAT"] >= 30 and checked["SAT"] >= 60, checked


def _partition_witness(k_sub, j, index, guard):
    lens = [1] * k_sub
    if guard != "le":
        lens[(j + 1) % k_sub if guard == "next" else (j - 1) % k_sub] = 3
    wit = {f"len{i}": lens[i] for i in range(k_sub)}
    wit["S"] = sum(lens)
    if index == "t":
        wit["t"] = 1
    else:
        wit.update(t=1, W=1, i=0)
    return wit


def test_family_partition_labels_by_brute_force():
    """partition_query for k_sub = 2..4 parts, every target part, both index
    forms and all four guards: the correct guard is UNSAT at the partition
    level, each buggy guard SAT (and the allocation-level test of the
    one-past-the-end guard UNSAT for a non-last part: Fig. 3's contrast).
    Part lengths have 2 bits and the other inputs 3, wide enough for the
    witness (a neighbour of length 3, the allocation k_sub + 2 elements);
    the batch's 20-bit inputs hold it for every k_sub."""
    n = 0
    for k_sub in (2, 3, 4):
        width, lens_w = 3, 2
        for j in range(k_sub):
            for index in ("t", "tw"):
                for guard in ("lt", "le", "next", "prev"):
                    q = partition_query(width, lens_w, k_sub, j, index, guard)
                    if q.input_bits > 22:
                        continue
                    want = "UNSAT" if guard == "lt" else "SAT"
                    assert _bf(q) == want, (k_sub, j, index, guard)
                    if want == "SAT":
                        wit = _partition_witness(k_sub, j, index, guard)
                        assert query_ref.int_eval(q, _named(q, wit))
                    n += 1
                if j < k_sub - 1:
                    qa = partition_query(width, lens_w, k_sub, j, "t", "le", level="allocation")
                    assert _bf(qa) == "UNSAT", (k_sub, j)
    assert n >= 60


@pytest.mark.parametrize("width", [2, 3, 4])
def test_family_lower_bound_labels_by_brute_force(width):
    for h in range(1, min(8, (1 << width) - 1) + 1):
        for s in (1, 2, 4, 8):
            assert _bf(oob_lower_1d(width, "ge", h, scale=s)) == "UNSAT"
            for guard, wit in (("none", dict(blockDim=1, blockIdx=0, threadIdx=0)),
                               ("ge_off", dict(blockDim=h, blockIdx=0, threadIdx=h - 1))):
                q = oob_lower_1d(width, guard, h, scale=s)
                assert _bf(q) == "SAT"
                if h < (1 << width):
                    assert query_ref.int_eval(q, _named(q, wit))


@pytest.mark.parametrize("m", [4, 5])
def test_family_wrap_labels_by_brute_force(m):
    """The machine-integer batch's rule: a guarded access with w-bit inputs
    and element size s is SAT with m-bit arithmetic iff s * 2^w > 2^m."""
    for width in range(max(1, m - 3), m + 1):
        for s in (1, 2, 4, 8):
            q = oob_1d(width, "lt", scale=s, header=0)
            want = "SAT" if s * (1 << width) > (1 << m) else "UNSAT"
            assert query_ref.wrap_bruteforce(q, m)[0] == want, (m, width, s)


def test_full_width_batches_follow_the_pinned_rules():
    """Every query of the full-width batches is an instance of a family
    pinned above, and its label is the family's rule for its variant."""
    for g in w.batch_1d():
        assert g.label == ("UNSAT" if "_lt_" in g.query.name else "SAT")
    for g in w.batch_2d(n=512):
        assert g.label == ("UNSAT" if g.kind == "guarded_2d" else "SAT")
    for g in w.partition_batch(n=256):
        assert g.label == ("UNSAT" if g.query.name.endswith("_lt") else "SAT")
    for g in w.batch_lower(n=128):
        assert g.label == ("UNSAT" if g.kind == "lower_guarded" else "SAT")
    for g in w.batch_wrap(n=64, m=32):
        s = int(g.query.name.rsplit("_s", 1)[1])
        wd = int(g.query.name.split("_w")[1].split("_")[0])
        assert g.label == ("SAT" if s * (1 << wd) > (1 << 32) else "UNSAT")


# ---------------------------------------------------------------- DPLL without the root check

@pytest.mark.parametrize("width", [2, 3, 4, 5, 6])
def test_guarded_single_access_refuted_by_dpll(width):
    """The fixed fact (a guarded idx < N access into N elements is UNSAT),
    reached by the oracle's own encoding and plain DPLL, the root check not
    consulted; the unguarded and off-by-one accesses are SAT the same way."""
    cnf, inputs = query_ref.encode(oob_1d(width, "lt", scale=4, header=0))
    assert cnf_ref.solve(cnf, 50_000_000)[0] == "UNSAT"
    for guard in ("none", "le"):
        q = oob_1d(width, guard, scale=4, header=0)
        cnf, inputs = query_ref.encode(q)
        v, model, _ = cnf_ref.solve(cnf)
        assert v == "SAT" and query_ref.int_eval(q, query_ref.decode_inputs(model, inputs))


@pytest.mark.parametrize("width", [2, 3, 4])
def test_guarded_1d_batch_shapes_refuted_by_dpll(width):
    """The 1-D batch's guarded shape with every element size and headers,
    refuted through the oracle's CNF by DPLL alone."""
    for s in (1, 2, 4, 8):
        for c in (0, 3, 16):
            cnf, _ = query_ref.encode(oob_1d(width, "lt", scale=s, header=c))
            assert cnf_ref.solve(cnf, 50_000_000)[0] == "UNSAT", (width, s, c)


def test_guarded_2d_shapes_refuted_by_dpll():
    """Correct 2-D guards through the multiplier, refuted by DPLL alone."""
    for mult, sep in ((1, False), (1, True), (2, False)):
        cnf, _ = query_ref.encode(oob_2d(2, "ok", mult, 2, 1, sep))
        assert cnf_ref.solve(cnf, 50_000_000)[0] == "UNSAT", (mult, sep)


def test_component_closed_form_matches_oracle_leaf():
    """The closed-form count and smallest index of the component formulas
    that the GPU test uses at 31..38 active variables equal the oracle's
    canonical leaf where #DPLL still finishes (10..18 variables)."""
    from tests.test_gpu_parity import _component_cnf
    for nv in (10, 12, 14, 16, 18):
        rng = np.random.Generator(np.random.PCG64(700 + nv))
        cnf, count, first = _component_cnf(nv, rng, f"comp{nv}")
        lf = cnf_ref.leaf(cnf, [])
        assert (lf["f"], lf["m"], lf["count"], lf["first"]) == (nv, 0, count, first)
