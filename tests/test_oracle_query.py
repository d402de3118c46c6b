"""Pins of the exact-integer query oracle: the paper's worked examples
(Sec. 3 and Sec. 4), the fixed facts about guarded and unguarded accesses,
closed-form counts, and exhaustive agreement between the oracle's own CNF
encoding and brute force over every input tuple.  CPU only."""
import numpy as np
import pytest

import workloads as w
from oracle import cnf_ref, query_ref
from tests.querygen import random_query
from workloads import oob_2d, batch_2d, Query, single_access, batch_1d, oob_1d, partition_query


# ---------------------------------------------------------------- worked examples

def _adv_cubature(wc=3, wn=3):
    """Fig. 1: id = threadIdx.y*16 + threadIdx.x in a 16x16 block; the
    buffer holds (cubN+1)^3 * Nelements * 3 elements."""
    q = Query("advCubature")
    cubN, nel = q.var("cubN", wc), q.var("Nelements", wn)
    tx, ty = q.var("tidx", 4), q.var("tidy", 4)      # ids below the 16x16 block
    q.require(tx < 16)
    q.require(ty < 16)
    cubNp = (cubN + 1) * (cubN + 1) * (cubN + 1)
    size = cubNp * nel * 3
    idx = ty * 16 + tx
    q.require(idx >= size)
    return q


def test_t1_adv_cubature_input_dependent_oob():
    q = _adv_cubature()
    # the paper's input: cubN = Nelements = 1 gives 24 elements, id up to 255
    assert query_ref.int_eval_named(q, dict(cubN=1, Nelements=1, tidx=15, tidy=15))
    vals = query_ref.int_eval_nodes(q, [1, 1, 15, 15])
    assert 24 in vals and 255 in vals
    v, wit, _ = query_ref.decide(q)
    assert v == "SAT" and query_ref.int_eval(q, wit)
    assert query_ref.int_bruteforce(q)[0] == "SAT"


def _saxpy(wm=6):
    """Fig. 5: index = threadIdx.x + blockDim.x*blockIdx.x with 512-thread
    blocks, gridDim = multiples, allocation multiples*512 elements."""
    q = Query("saxpy")
    mult, bid, tid = q.var("multiples", wm), q.var("blockIdx", wm), q.var("threadIdx", 9)
    q.require(tid < 512)
    q.require(bid < mult)
    q.require(tid + bid * 512 >= mult * 512)
    return q


def test_t2_saxpy_bound_by_relation():
    q = _saxpy()
    assert query_ref.int_bruteforce(q)[0] == "UNSAT"
    assert query_ref.decide(q)[0] == "UNSAT"


def test_t3_push_node_loaded_index():
    """Fig. 2: the index is a value loaded from memory (an unknown)."""
    q = Query("pushNode")
    numv, tid, bid, bdim = (q.var(n, 5) for n in ("numv", "tid", "bid", "bdim"))
    neighbor = q.var("neighbor", 5)
    q.require(tid < bdim)
    q.require(bid * bdim + tid < numv)          # if (i < numv)
    q.require(neighbor >= numv)                 # data1 has numv entries
    v, wit, _ = query_ref.decide(q)
    assert v == "SAT" and query_ref.int_eval(q, wit)


def test_t4_intra_allocation_partition():
    """Fig. 3 / Sec. 6.1: an index pushed one past a non-last partition
    stays inside the allocation yet leaves its partition."""
    for k_sub, j in ((3, 1), (2, 0)):
        alloc = partition_query(4, 3, k_sub, j, "t", "le", level="allocation")
        part = partition_query(4, 3, k_sub, j, "t", "le", level="partition")
        assert query_ref.int_bruteforce(alloc)[0] == "UNSAT"
        assert query_ref.int_bruteforce(part)[0] == "SAT"
        ok = partition_query(4, 3, k_sub, j, "t", "lt", level="partition")
        assert query_ref.int_bruteforce(ok)[0] == "UNSAT"
        assert query_ref.root_check(ok) == "UNSAT"


def test_t5_local_buffer_loop_bound():
    """Fig. 4: local arrays of rd entries indexed by a loop i < rd."""
    for guard, want in (("lt", "UNSAT"), ("le", "SAT")):
        q = Query("kalman")
        rd, i = q.var("rd", 6), q.var("i", 6)
        q.require(i < rd if guard == "lt" else i <= rd)
        q.require(i >= rd)
        assert query_ref.int_bruteforce(q)[0] == want
        assert query_ref.decide(q)[0] == want
        if want == "SAT":
            assert query_ref.int_eval_named(q, dict(rd=5, i=5))


def test_t6_lu_decomposition_multiple_of_16():
    """Sec. 6.1: the OOB shows only when N is not a multiple of 16 (grid of
    ceil(N/16) blocks of 16 threads, no guard)."""
    q = Query("lud")
    N, bid, tid = q.var("N", 7), q.var("bid", 4), q.var("tid", 4)
    q.require(bid < (N + 15) // 16)
    q.require(tid < 16)
    q.require(bid * 16 + tid >= N)
    verdict, cnt, _ = query_ref.int_bruteforce(q)
    assert verdict == "SAT"
    for n in range(0, 128, 16):          # every multiple of 16 is safe
        for b in range(16):
            for t in range(16):
                assert not query_ref.int_eval(q, [n, b, t]) if b < (n + 15) // 16 else True
    # count: for N = 16a + r (r > 0) exactly the 16 - r threads of the
    # last block past N go out of bounds
    want = sum(16 - (n % 16) for n in range(128) if n % 16)
    assert cnt == want
    v, wit, _ = query_ref.decide(q)
    assert v == "SAT" and wit[0] % 16 != 0


# ---------------------------------------------------------------- fixed facts

def test_guarded_access_is_unsat_and_unguarded_sat():
    assert query_ref.root_check(single_access("lt").query) == "UNSAT"
    for variant in ("none", "le"):
        g = single_access(variant)
        assert query_ref.int_eval_named(g.query, g.witness)
        v, wit, _ = query_ref.decide(g.query)
        assert v == "SAT" and query_ref.int_eval(g.query, wit)


@pytest.mark.parametrize("w", [2, 3, 4, 5])
def test_unguarded_count_closed_form(w):
    """#{(N, bdim, bid, tid) : tid < bdim, bid*bdim + tid >= N}: for each
    (bdim, tid, bid) the admissible N are 0 .. min(2^w - 1, idx)."""
    top = 1 << w
    b = np.arange(top)[:, None, None]
    t = np.arange(top)[None, :, None]
    i = np.arange(top)[None, None, :]
    idx = i * b + t
    want = int(np.where(t < b, np.minimum(top, idx + 1), 0).sum())
    q = oob_1d(w, "none", scale=4)
    assert query_ref.int_bruteforce(q)[1] == want
    if w <= 3:
        cnf, _ = query_ref.encode(q)
        assert cnf_ref.count(cnf) == want


@pytest.mark.parametrize("w", [2, 3, 4])
def test_guarded_small_widths_unsat(w):
    for s, c in ((1, 0), (4, 3), (8, 16)):
        q = oob_1d(w, "lt", scale=s, header=c)
        assert query_ref.int_bruteforce(q)[0] == "UNSAT"
        cnf, _ = query_ref.encode(q)
        assert cnf_ref.solve(cnf)[0] == "UNSAT"


def test_batch_1d_labels_by_construction():
    gens = batch_1d()
    assert sum(g.label == "UNSAT" for g in gens) == 128
    for g in gens:
        if g.label == "UNSAT":
            assert query_ref.root_check(g.query) == "UNSAT"
        else:
            assert query_ref.int_eval_named(g.query, g.witness)
            assert query_ref.root_check(g.query) is None


@pytest.mark.parametrize("w", [2, 3, 4])
def test_lower_bound_small_widths(w):
    """Lower-bound stencil reads buf[idx - h] against exhaustive integer
    search: the guard idx >= h leaves no input below the buffer, the guard
    off by one and no guard do; the oracle's encoding agrees at w <= 3."""
    from workloads import oob_lower_1d
    for h in (1, 2, 3):
        if h >= (1 << w):
            continue
        for s in (1, 4):
            for g, want in (("ge", "UNSAT"), ("ge_off", "SAT"), ("none", "SAT")):
                q = oob_lower_1d(w, g, h, scale=s)
                assert query_ref.int_bruteforce(q)[0] == want, (w, h, s, g)
                assert query_ref.decide(q)[0] == want, (w, h, s, g)
                if w <= 3:
                    cnf, _ = query_ref.encode(q)
                    assert cnf_ref.solve(cnf)[0] == want


def test_lower_bound_unguarded_count_closed_form():
    """#{(bdim, bid, tid) : tid < bdim, bid*bdim + tid < h} over 3-bit
    inputs, counted directly, equals the brute-force count of the unguarded
    lower-bound query (every admissible idx below h reads below the buffer)."""
    from workloads import oob_lower_1d
    top, h = 8, 3
    b = np.arange(top)[:, None, None]
    i = np.arange(top)[None, :, None]
    t = np.arange(top)[None, None, :]
    want = int(((t < b) & (i * b + t < h)).sum())
    q = oob_lower_1d(3, "none", h, scale=4)
    assert query_ref.int_bruteforce(q)[1] == want


def test_lower_bound_labels_by_construction():
    from workloads import batch_lower
    gens = batch_lower(n=96)
    assert sum(g.label == "UNSAT" for g in gens) == 48
    for g in gens:
        if g.label == "UNSAT":
            assert query_ref.root_check(g.query) == "UNSAT", g.query.name
        else:
            assert query_ref.int_eval_named(g.query, g.witness), g.query.name
            assert query_ref.root_check(g.query) is None


# ---------------------------------------------------------------- machine integers

@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_wrap_unsigned_overflow_closed_form(m):
    """a + b < a (unsigned) holds exactly when a + b >= 2^m, i.e. for
    sum_a a = 2^m (2^m - 1) / 2 pairs; never with exact integers."""
    q = Query("ovf")
    a, b = q.var("a", m), q.var("b", m)
    q.require(a + b < a)
    assert query_ref.wrap_bruteforce(q, m)[1] == (1 << m) * ((1 << m) - 1) // 2
    assert query_ref.int_bruteforce(q)[0] == "UNSAT"


def test_wrap_matches_exact_when_nothing_overflows():
    """With no subtraction and m far above every magnitude the machine
    integers are the integers: both brute forces count the same tuples."""
    rng = np.random.Generator(np.random.PCG64(401))
    checked = 0
    for i in range(80):
        q = random_query(rng, max_bits=9, ops=("add", "mul", "shl", "udiv", "urem", "const"), name=f"n{i}")
        if max(query_ref._magnitude_bounds(q) + [0]) >= (1 << 59):
            continue
        assert query_ref.wrap_bruteforce(q, 60)[1] == query_ref.int_bruteforce(q)[1], q.nodes
        checked += 1
    assert checked >= 40


def test_wrap_labels_by_construction_small():
    """The wrap-around workload at m = 5 (inputs of 3..5 bits): every label
    equals exhaustive search with 5-bit machine integers, and each SAT
    witness satisfies that evaluation; with exact integers all are UNSAT."""
    gens = w.batch_wrap(n=48, m=5, wspan=2)
    assert {g.label for g in gens} == {"SAT", "UNSAT"}
    for g in gens:
        assert query_ref.wrap_bruteforce(g.query, 5)[0] == g.label, g.query.name
        assert query_ref.int_bruteforce(g.query)[0] == "UNSAT"
        if g.label == "SAT":
            assert query_ref.wrap_eval(g.query, [g.witness[n] for n in g.query.var_names], 5)


def test_batch_2d_labels_by_construction():
    """Correct 2-D guards are UNSAT by the chain row*ld + col <= (R-1)*ld +
    (C-1) < R*ld (C <= ld); the root check must find it through the
    product lemma ld*(R - 1 - row) >= 0.  Buggy ones carry witnesses."""
    gens = batch_2d(n=600)
    assert sum(g.label == "UNSAT" for g in gens) == 300
    kinds = set()
    for g in gens:
        kinds.add(g.kind)
        if g.label == "UNSAT":
            assert query_ref.root_check(g.query) == "UNSAT", g.query.name
        else:
            assert query_ref.int_eval_named(g.query, g.witness), g.query.name
            assert query_ref.root_check(g.query) is None, g.query.name
    assert len(kinds) == 6


@pytest.mark.parametrize("w", [2, 3])
def test_oob_2d_small_widths_match_brute_force(w):
    """At widths the brute force covers, every 2-D variant's verdict and the
    root check agree with exhaustive integer evaluation."""
    for guard in ("ok", "no_row", "no_col", "row_le", "col_le", "ld_free"):
        for mult, sep in ((1, False), (1, True), (2, False)):
            if guard != "ok" and sep:
                continue
            q = oob_2d(w, guard, mult, 2, 1, sep)
            if q.input_bits > 20:
                continue
            verdict = query_ref.int_bruteforce(q)[0]
            assert verdict == ("UNSAT" if guard == "ok" else "SAT"), (guard, mult, sep)
            rc = query_ref.root_check(q)
            assert rc is None or verdict == "UNSAT"


def test_fourier_motzkin_textbook_systems():
    fm = query_ref.fm_infeasible
    # x >= 1, y >= 1, x + y <= 1: infeasible
    assert fm([({"x": 1}, -1), ({"y": 1}, -1), ({"x": -1, "y": -1}, 1)])
    # 2x >= 1, 2x <= 1: x = 1/2 is a rational solution (integers aside)
    assert fm([({"x": 2}, -1), ({"x": -2}, 1)]) is False
    # x - y >= 0, y - z >= 0, z - x >= 1: a cycle that must grow
    assert fm([({"x": 1, "y": -1}, 0), ({"y": 1, "z": -1}, 0), ({"z": 1, "x": -1}, -1)])
    # the same cycle closed with 0: feasible (x = y = z)
    assert fm([({"x": 1, "y": -1}, 0), ({"y": 1, "z": -1}, 0), ({"z": 1, "x": -1}, 0)]) is False
    # 3x + 2y >= 7, x <= 1, y <= 2: max 3 + 4 = 7 -> feasible at (1, 2)
    sys_ = [({"x": 3, "y": 2}, -7), ({"x": -1}, 1), ({"y": -1}, 2)]
    assert fm(sys_) is False
    sys_[0] = ({"x": 3, "y": 2}, -8)
    assert fm(sys_)


def test_batch_1d_sat_decided_at_full_width():
    gens = [g for g in batch_1d() if g.label == "SAT"][:12]
    for g in gens:
        v, wit, _ = query_ref.decide(g.query)
        assert v == "SAT" and query_ref.int_eval(g.query, wit), g.query.name


# ---------------------------------------------------------------- encoder + root check

def test_encoder_counts_match_brute_force():
    rng = np.random.Generator(np.random.PCG64(21))
    for i in range(150):
        q = random_query(rng, max_bits=9, name=f"r{i}")
        verdict, cnt, _ = query_ref.int_bruteforce(q)
        cnf, inputs = query_ref.encode(q)
        assert cnf_ref.count(cnf) == cnt, q.nodes
        v, model, _ = cnf_ref.solve(cnf)
        assert v == verdict
        if model is not None:
            assert query_ref.int_eval(q, query_ref.decode_inputs(model, inputs))


def test_root_check_is_sound():
    rng = np.random.Generator(np.random.PCG64(22))
    hits = 0
    for i in range(400):
        q = random_query(rng, max_bits=10, ops=("add", "sub", "mul", "shl", "const"))
        if query_ref.root_check(q) == "UNSAT":
            hits += 1
            assert query_ref.int_bruteforce(q)[0] == "UNSAT", q.nodes
    assert hits > 10
