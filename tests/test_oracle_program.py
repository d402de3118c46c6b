"""Pins of the program interpreter (oracle/program_ref.py): verdicts and
event counts of the example programs, worked out by hand from their text.

An event is one (input assignment, thread, loop iteration) at which an access
leaves its data structure.  Each count below is a closed form over the
inputs' ranges, derived from the program's arithmetic, not from running it.
"""
import pytest

from oracle import program_ref as pr
import workloads.program as P


@pytest.fixture(scope="module")
def results():
    return {p.name: (p, pr.brute_force(p, lower=True)) for p in P.examples()}


def _out(res, key):
    return res[key][0], res[key][2]


def test_guarded_grid(results):
    p, r = results["guarded_grid"]
    # scale: i < len guards both accesses of an n-element buffer
    for ai in (0, 1):
        assert _out(r, (0, "scale", ai, "upper")) == (False, 0)
    # scale_le: i <= len lets thread i = n through whenever the rounded-up
    # grid has it, i.e. n is not a multiple of 32: 256 - 8 values of n
    assert _out(r, (1, "scale_le", 0, "upper")) == (True, 256 - 8)
    assert not any(r[k][0] for k in r if k[3] == "lower")


def test_asserted_multiple(results):
    p, r = results["asserted_multiple"]
    assert _out(r, (0, "copy", 0, "upper")) == (False, 0)
    assert _out(r, (0, "copy", 1, "upper")) == (False, 0)   # b[i + 8], b has n + 8
    # b[i + 9] leaves for i = n - 1 only; n a positive multiple of 16 below 128
    assert _out(r, (0, "copy", 2, "upper")) == (True, 7)


def test_shm_partitions(results):
    p, r = results["shm_partitions"]
    # parts: base [0, m), vals [m, 2m), tail [2m, 2m + extra); threads t < m
    assert _out(r, (0, "kv", 0, "upper")) == (False, 0)        # base[t]
    assert _out(r, (0, "kv", 1, "upper")) == (False, 0)        # vals[t]
    assert _out(r, (0, "kv", 2, "upper")) == (True, 31 * 8)    # vals[t + 1]: t = m - 1, m >= 1
    tail = sum(max(0, m - extra) for m in range(32) for extra in range(8))
    assert _out(r, (0, "kv", 3, "upper")) == (True, tail)      # tail[t]: t >= extra
    assert _out(r, (0, "kv", 4, "upper")) == (False, 0)        # p[t], p has m
    assert not any(r[k][0] for k in r if k[3] == "lower")


def test_tile_halo(results):
    p, r = results["tile_halo"]
    # tile has 240 elements; (y + 1) * 16 + x >= 240 needs y = 14, so h = 15:
    # every x < w, summed over w
    assert _out(r, (0, "blur", 0, "upper")) == (False, 0)
    assert _out(r, (0, "blur", 1, "upper")) == (True, sum(range(16)))
    # the else-branch read p[y*w + x - 1] runs for x = w - 1 and is negative
    # only for w = 1, y = 0: one thread for each h = 1..15
    assert _out(r, (0, "blur", 4, "lower")) == (True, 15)
    for ai in (2, 3, 4):
        assert _out(r, (0, "blur", ai, "upper")) == (False, 0)
    for ai in (0, 1, 2, 3):
        assert _out(r, (0, "blur", ai, "lower")) == (False, 0)


def test_strided_loop(results):
    p, r = results["strided_loop"]
    assert _out(r, (0, "rows", 0, "upper")) == (False, 0)
    # b[row*k + j + 1] with row = n - 1, j = k - 1; rows 0..7 exist, so n = 1..8
    assert _out(r, (0, "rows", 1, "upper")) == (True, 8 * 7)
    assert _out(r, (0, "rows", 2, "upper")) == (False, 0)      # acc[threadIdx.x]


def test_stencil_left(results):
    p, r = results["stencil_left"]
    assert _out(r, (0, "left", 0, "lower")) == (True, 63)      # i = 0 for every n >= 1
    assert _out(r, (0, "left", 1, "lower")) == (False, 0)      # guarded by i >= 1
    assert _out(r, (0, "left", 0, "upper")) == (False, 0)


def test_witness_replay(results):
    # the interpreter's own first witnesses go out; a thread that stays in
    # bounds does not
    for name, (p, r) in results.items():
        for key, (out, wit, _) in r.items():
            if not out:
                continue
            inputs, bid, tid, loops = wit
            vals = dict(inputs)
            for i, a in enumerate("xyz"):
                vals[f"blockIdx.{a}"], vals[f"threadIdx.{a}"] = bid[i], tid[i]
            vals.update({f"for:{k}": v for k, v in loops.items()})
            assert pr.witness_goes_out(p, key, vals), (name, key)
    p, _ = results["guarded_grid"]
    assert pr.witness_goes_out(p, (1, "scale_le", 0, "upper"), {"n": 5, "threadIdx.x": 5})
    assert not pr.witness_goes_out(p, (1, "scale_le", 0, "upper"), {"n": 5, "threadIdx.x": 4})
    assert not pr.witness_goes_out(p, (1, "scale_le", 0, "upper"), {"n": 32, "threadIdx.x": 32})


def test_failed_assert_stops_the_launches():
    p = P.parse("""
        input n : 3
        malloc A = n
        assert n >= 8
        launch k grid(1) block(4) args(A)
        kernel k(a) { load a[threadIdx.x] }
    """, "never")
    assert not pr.brute_force(p)[(0, "k", 0, "upper")][0]
