"""Throughput of the OOB-query decision path on one MI355X.

One step = the whole path for one batch: query DAGs -> normalisation and
Tseitin CNF (host) -> cube splitting (host) -> device unit propagation and
bit-sliced leaf evaluation (gfx950) -> verified verdicts and witnesses.

Default workload (the largest single-GPU batch): 4096 seeded 2-D row-major
accesses of uneven width (inputs of 8-24 bits, one to three multipliers in
the offset, guards row < R and col < C), 2048 correct (UNSAT) and 2048 buggy
(SAT), decided in one call per step with autotuned options (cube depth k,
work-item size, leaves per round, grid, leaf tile, HIP graphs).

Prints one JSON line: queries decided per second over the timed steps for
the headline cube ordering, the same for every ordering (static, learned,
word) with its agreement, the roofline of the dominant kernel (HIP events
bracketing each dispatch, on the stream the kernel runs on), microbenchmark
peaks of this GPU, and the CPU oracle timed on this host's cores.  Every
step's verdicts are checked against the generators' labels (pinned by
exhaustive search in the CPU tests); the CPU-baseline leg re-decides a
sample with the oracle and re-checks every witness exactly.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# int32 VALU lane-ops/s: 256 CU x 128 lanes per clock x 2.4 GHz.  The lane
# rate is the one the fp32 vector peak (157.3 TFLOP/s, 2 flops per FMA)
# implies, and the microbenchmark's chains of separate v_xor_b32 / v_add_u32
# reach 89 % of it on this GPU (a 4-SIMD x 16-lane count, 39.3 T, is below
# what the hardware measurably issues)
PEAK_INT32_TOPS = 78.6432
PEAK_HBM_GBS = 8000.0
# per evaluated clause-block (one residual clause against 4096 assignments):
# the 64-bit AND of the clause's satisfaction word into each of the 64 lanes'
# accumulators = 64 lanes x 2 int32 ops
OPS_PER_CLAUSE_BLOCK = 128

# HBM bytes per launch from two rocprofv3 counter passes (FETCH_SIZE /
# 0.5 + WRITE_SIZE, both scaled by what they read for a device copy of known
# size), valid only for the kernel source, workload and options they were
# taken on (profiles/fix_kernel_batch2d_4096q.md)
MEASURED_TRAFFIC = {
    'batch_2d:f845fbcdbe9473c6:{"chunk_log2": 8, "form": "word", "graph": false, "grid": 4096, "k": 30, '
    '"leaves_per_round": 1, "max_cubes": 20000, "max_residual": 4096, "scorer": "word"}': {
        "fix_kernel": 948268098, "leaf_kernel": 2064567},
}

# The autotuner's choices for this bench's batches on MI355X (gfx950), as
# scuba_tune_cache_save wrote them after a tuning run of this script; loaded
# before tuning so that every run times (and the profiles cover) the same
# options.  Batches it does not cover, and other architectures, tune live.
TUNE_CACHE = os.path.join(ROOT, "paper_2601_21552_amd", "tune_cache.jsonl")

# leaf-evaluation variants of the leaf profile (solve options)
LEAF_VARIANTS = {"scalar": {}, "vector": {"leaf": "vector"}, "lds": {"leaf": "lds"}}

# learned ordering: candidates scored per decision node, and the levels
# below a scored node that reuse its ranking
LEARNED_CANDIDATES = 16
LEARNED_RESCORE = 4
LEARNED_RESCORE_ACCESS = 128

WORKLOADS = {
    "batch_2d": ("4096 seeded 2-D OOB queries of uneven width: inputs 8-24 bits, 1-3 multipliers per "
                 "offset (row = by*bdy+ty, col = bx*bdx+tx), offset (row*ld+col)*s+c vs size R*ld*s+c, "
                 "2048 guarded (UNSAT) / 2048 buggy (SAT); one decide call per step, autotuned (the persisted "
                 "choices when present), HIP graphs"),
    "batch_1d": ("256 seeded 1-D OOB queries, widths 8-16 bits, s in {1,2,4,8}, c in 0..16, "
                 "128 guarded (UNSAT) / 64 unguarded + 64 off-by-one (SAT); k=30"),
    "single": "one 12-bit guarded idx<N query (UNSAT), k=30",
}
MAX_CUBES = {"batch_2d": 20000, "batch_1d": 100000, "single": 100000}


def log(m):
    print(m, file=sys.stderr, flush=True)


def make_batch(workload: str):
    import workloads as w
    if workload == "single":
        return [w.single_access("lt")]
    if workload == "batch_1d":
        return w.batch_1d()
    return w.batch_2d()


def train_scorer(ctx, batches, k, epochs, seed, candidates=32, depth=24):
    """The learned scorer trained on the splitter's own traces of `batches`
    (CNF handles), forward / backward / Adam in the library's kernels."""
    from paper_2601_21552_amd import train
    f, lab, nodes = train.collect(ctx, batches, k=k, candidates=candidates, depth=depth,
                                  max_cubes=2000)
    mlp, hist = train.train(ctx, f, train.node_targets(lab, nodes), epochs=epochs, seed=seed)
    return mlp, {"rows": int(len(lab)), "epochs": epochs, "loss_first": round(hist[0], 4),
                 "loss_last": round(hist[-1], 4)}


def decide_stats(ctx, cnf, n, labels=None, **opts):
    """One decide call: wall ms, verdict counts, leaves and cubes."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.decide(cnf, **opts)
    ms = 1000.0 * (time.perf_counter() - t0)
    tm = res.timing()
    out = {"ms": round(ms, 2), "SAT": 0, "UNSAT": 0, "UNKNOWN": 0, "leaves": 0, "cubes": 0,
           "split_ms": round(tm["split"], 2), "kernels_ms": round(tm["kernels"], 2)}
    if tm["score_passes"]:
        out.update(score_passes=int(tm["score_passes"]), score_rows=int(tm["score_rows"]),
                   score_device_ms=round(tm["score_device"], 2))
    verdicts = []
    for i in range(n):
        r = res.result(i)
        verdicts.append(r["verdict"])
        out[r["verdict"]] += 1
        out["leaves"] += r["leaves_sent"]
        out["cubes"] += r["cubes_total"]
        if r["verdict"] == "SAT":
            assert r["witness_checked"]
    if labels is not None:
        wrong = sum(v != "UNKNOWN" and v != l for v, l in zip(verdicts, labels))
        assert wrong == 0, "a verdict contradicts the generator's label"
        out["agree"] = sum(v == l for v, l in zip(verdicts, labels)) / n
    return out, verdicts


class Steps:
    """Timed steps of the whole path on one batch: bit-blast of the packed
    query DAGs, then one decide call with fixed options."""

    def __init__(self, ctx, packed, gens, stream, args):
        self.ctx, self.packed, self.gens, self.stream, self.args = ctx, packed, gens, stream, args
        self.labels = [g.label for g in gens]

    def run(self, opts, steps=None, warmup=None):
        import torch
        ctx = self.ctx
        steps = self.args.steps if steps is None else steps
        warmup = self.args.warmup if warmup is None else warmup
        bb_ms = []

        def step():
            t0 = time.perf_counter()
            cnf = ctx.bitblast_packed(*self.packed)
            bb_ms.append(1000.0 * (time.perf_counter() - t0))
            return cnf, ctx.decide(cnf, stream=self.stream, **opts)

        # the first call of a fresh shape (graph captures included)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        first_ms = 1000.0 * (time.perf_counter() - t0)
        for _ in range(max(warmup - 1, 0)):
            step()
        torch.cuda.synchronize()
        bb_ms.clear()
        t0 = time.perf_counter()
        out, last_cnf = [], None
        for _ in range(steps):
            cnf, res = step()
            out.append(res)
            last_cnf = cnf   # a step's CNF is released when the next replaces it
            del cnf
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        agree, unknown = [], 0
        for res in out:
            vs = res.verdicts()
            wrong = sum(v != "UNKNOWN" and v != l for v, l in zip(vs, self.labels))
            assert wrong == 0, ("a verdict contradicts the generator's label", opts)
            agree.append(sum(v == l for v, l in zip(vs, self.labels)) / len(vs))
            unknown = sum(v == "UNKNOWN" for v in vs)
            for i, v in enumerate(vs):
                if v == "SAT":
                    assert res.result(i)["witness_checked"]
        return dict(ms_per_step=1000.0 * elapsed / steps, results=out, cnf=last_cnf,
                    first_ms=first_ms, agree=min(agree), unknown=unknown,
                    bitblast_ms=sorted(bb_ms)[len(bb_ms) // 2])


def kernel_accounting(steps: "Steps", run, traffic_key):
    """Per-kernel durations (HIP events bracketing each dispatch), launches
    and algorithmic work of a run's steps; the dominant kernel's roofline."""
    res_list, cnf = run["results"], run["cnf"]
    n = len(steps.gens)
    leaf_ms = up_ms = 0.0
    leaf_launches = up_launches = fix_launches = 0
    split_ms = verify_ms = 0.0
    for res in res_list:
        tm = res.timing()
        leaf_ms += tm["leaf"]
        up_ms += tm["up"]
        leaf_launches += int(tm["leaf_launches"])
        up_launches += int(tm["up_launches"])
        fix_launches += int(tm["fix_launches"])
        split_ms += tm["split"]
        verify_ms += tm["verify"]
    res = res_list[-1]
    k = len(res_list)
    detail = dict(decided_at_root=0, decided_on_device=0, unknown=0, leaves_sent=0, leaves_refuted=0,
                  blocks_evaluated=0, clause_blocks=0, word_ops=0)
    up_bytes = 0
    for i in range(n):
        r = res.result(i)
        detail["decided_at_root"] += r["how"] == "root"
        detail["decided_on_device"] += r["how"] == "device"
        detail["unknown"] += r["verdict"] == "UNKNOWN"
        for key in ("leaves_sent", "leaves_refuted", "blocks_evaluated", "clause_blocks", "word_ops"):
            detail[key] += r[key]
        if r["leaves_sent"]:
            v = cnf.sizes(i)
            # every cube sent reads its query's CSR CNF once: 4 (C + 1 + L) bytes
            up_bytes += r["leaves_sent"] * 4 * (v["n_clauses"] + 1 + v["n_lits"])
    last = res.timing()
    prop = ("fix_kernel" if fix_launches == up_launches else
            "up_kernel" if fix_launches == 0 else "up_kernel+fix_kernel")
    lpl = max(int(last["leaf_launches"]), 1)
    upl = max(int(last["up_launches"]), 1)
    kernels = {
        "leaf_kernel": dict(bound="alu", ms_step=leaf_ms / k, avg=leaf_ms / max(leaf_launches, 1),
                            per_launch=2 * detail["word_ops"] / lpl,
                            peak=PEAK_INT32_TOPS, unit="TOP/s (int32 lane-ops: 2 per 64-bit word op, "
                            "64 words x (|c|+1) per evaluated clause-block)", scale=1e12,
                            launches=leaf_launches / k,
                            clause_block_rate=OPS_PER_CLAUSE_BLOCK * detail["clause_blocks"] / lpl),
        # the propagation stage: fix_kernel when every cube carried the
        # host's fixpoint, up_kernel otherwise
        prop: dict(bound="hbm", ms_step=up_ms / k, avg=up_ms / max(up_launches, 1),
                   per_launch=up_bytes / upl, peak=PEAK_HBM_GBS,
                   unit="GB/s (each cube's CSR CNF read once)", scale=1e9, launches=up_launches / k),
    }
    dom = max(kernels, key=lambda x: kernels[x]["ms_step"])

    def line(name):
        kd = kernels[name]
        ach = kd["per_launch"] / (kd["avg"] * 1e-3) / kd["scale"] if kd["avg"] > 0 else 0.0
        tr = MEASURED_TRAFFIC.get(traffic_key, {}).get(name)
        out = {"kernel": name, "bound": kd["bound"], "achieved": round(ach, 4), "peak": kd["peak"],
               "unit": kd["unit"], "frac": round(ach / kd["peak"], 5), "traffic": tr,
               "avg_launch_ms": round(kd["avg"], 4), "launches_per_step": kd["launches"],
               "per_launch": kd["per_launch"]}
        if name == "leaf_kernel":
            out["clause_block_rate_tops"] = round(kd["clause_block_rate"] / (kd["avg"] * 1e-3) / 1e12, 4) \
                if kd["avg"] > 0 else 0.0
        return out
    roof = line(dom)
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    roof["other"] = line("leaf_kernel" if dom == prop else prop)
    detail.update(host_split_ms_per_step=round(split_ms / k, 3), verify_ms_per_step=round(verify_ms / k, 3),
                  leaf_kernel_ms_per_step=round(leaf_ms / k, 3), propagation_ms_per_step=round(up_ms / k, 3))
    return roof, detail


def traffic_key(workload, opts):
    src = os.path.join(ROOT, "paper_2601_21552_amd", "csrc", "device.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return f"{workload}:{sha}:{json.dumps(opts, sort_keys=True)}"


# ------------------------------------------------------------------ CPU baseline

def _oracle_decide(q):
    from oracle import query_ref
    return query_ref.decide(q)[0]


def _oracle_3sat(f):
    """The oracle's DPLL verdict on one raw formula (node budget 3e8)."""
    from oracle import cnf_ref
    return cnf_ref.solve(f, 300_000_000)[0]


DPLL_CNF_NODES = 20_000


def _oracle_dpll(arrs):
    """The oracle's C DPLL on one query's CNF bytes as the library emitted
    them (root-refuted queries have no CNF: UNSAT), with a node budget."""
    import numpy as np
    from oracle import cnf_ref
    from workloads.cnf import CNF
    n_vars, off, lits, root_unsat = arrs
    if root_unsat:
        return "UNSAT"
    return cnf_ref.solve(CNF(n_vars, np.asarray(off, np.uint64), np.asarray(lits, np.int32)),
                         DPLL_CNF_NODES)[0]


def cpu_baseline_leg(gens, cnf, path_verdicts, results_last):
    """The oracle as it stands, timed on this host: (1) the whole oracle
    (root check, own Tseitin encoding, C DPLL) on a stratified sample of the
    batch, on every core of this process's share and on one core; (2) the C
    DPLL alone on the library's own CNF bytes of the same sample (bit-blast
    is shared and timed on its own line).  Checks the oracle's verdicts
    against the path's, and every SAT witness of the path exactly."""
    from concurrent.futures import ProcessPoolExecutor
    from oracle import query_ref
    n = len(gens)
    # the process's CPU share (16 on a one-GPU machine); the pool is capped there
    cores = min(len(os.sched_getaffinity(0)), 16)
    m = min(n, 256)
    idx = [i * n // m for i in range(m)]
    sample = [gens[i].query for i in idx]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        ov = list(ex.map(_oracle_decide, sample, chunksize=2))
    dt_all = time.perf_counter() - t0
    log(f"cpu baseline: whole oracle on {m} queries, {cores} processes: {dt_all:.2f} s")
    one = idx[:max(m // 8, 1)]
    t0 = time.perf_counter()
    ov1 = [_oracle_decide(gens[i].query) for i in one]
    dt_one = time.perf_counter() - t0
    log(f"cpu baseline: whole oracle on {len(one)} queries, one core: {dt_one:.2f} s")
    agree = sum(a == path_verdicts[i] for a, i in zip(ov, idx)) / m
    unknown = sum(a == "UNKNOWN" for a in ov)
    assert all(a == path_verdicts[i] for a, i in zip(ov1, one))
    # the C DPLL on the library's CNF bytes
    # its own smaller sample (every n/64-th query)
    md = min(n, 64)
    idx_d = [i * n // md for i in range(md)]
    one_d = idx_d[:max(md // 8, 1)]
    arrs = []
    for i in idx_d:
        v = cnf.view(i)
        arrs.append((v["n_vars"], v["clause_off"], v["lits"], bool(v["root_unsat"])))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        dv = list(ex.map(_oracle_dpll, arrs, chunksize=2))
    dt_dpll = time.perf_counter() - t0
    log(f"cpu baseline: DPLL on the library's CNF bytes, {md} queries, {cores} processes: {dt_dpll:.2f} s")
    t0 = time.perf_counter()
    dv1 = [_oracle_dpll(a) for a in arrs[:len(one_d)]]
    dt_dpll1 = time.perf_counter() - t0
    log(f"cpu baseline: DPLL on the library's CNF bytes, {len(one_d)} queries, one core: {dt_dpll1:.2f} s")
    decided = [(a, i) for a, i in zip(dv, idx_d) if a != "UNKNOWN"]
    dpll_agree = (sum(a == path_verdicts[i] for a, i in decided) / len(decided)) if decided else None
    assert dv1 == dv[:len(one_d)]
    # every SAT witness of the last timed step, by the exact definition
    for i, g in enumerate(gens):
        if path_verdicts[i] == "SAT":
            assert query_ref.int_eval(g.query, results_last.witness(i, g.query.n_vars))
    return {
        "value": round(m / dt_all, 3), "unit": "queries/s", "cores": cores, "kind": "oracle",
        "sample": (f"{m} of the {n} queries (every {n // m}th), the whole oracle per query (root check, "
                   f"own Tseitin encoding, C DPLL) in {cores} processes: {dt_all:.2f} s wall; the pool is "
                   "capped at 16, this process's CPU share on a one-GPU box"),
        "one_core": {"value": round(len(one) / dt_one, 3), "queries": len(one), "seconds": round(dt_one, 2)},
        "dpll_on_library_cnf": {
            "value": round(md / dt_dpll, 3), "cores": cores, "one_core_value": round(len(one_d) / dt_dpll1, 3),
            "queries": md, "one_core_queries": len(one_d),
            "note": f"C DPLL on the CNF bytes the library bit-blasted (shared bit-blast excluded; queries the "
                    f"root stage refuted have no CNF and count as decided), at most {DPLL_CNF_NODES} nodes per "
                    "query (static MOMs branching without the word-level bounds can run for minutes on one "
                    "SAT query); agreement over the queries it decided",
            "unknown": sum(a == "UNKNOWN" for a in dv),
            "agreement": dpll_agree},
        "oracle_agreement": agree, "oracle_unknown": unknown,
    }


# ------------------------------------------------------------------ other legs

def gain_legs(ctx, mlp_q, mlp_s_info, args):
    """Learned vs static on samples of the random 3-SAT sets (scorer trained
    on disjoint-seed instances) at every n, with autotuned k, and the
    partition queries; the smaller access workloads and the front-end."""
    import workloads as w
    from oracle import cnf_ref
    out = {}
    mlp_s, info = mlp_s_info
    out["random3sat_scorer"] = info
    # seeded samples of the 2500 instances per n; the static ordering split
    # on the device and on the host, the learned ordering on the host (its
    # scorer runs between host decisions); k autotuned on the sample
    per_n = {100: 256, 150: 128, 200: 32, 250: 16}
    learned_n = {100: 256, 150: 64, 200: 8, 250: 4}
    host_n = {100: 256, 150: 64, 200: 8, 250: 4}
    oracle_n = {100: 32, 150: 8, 200: 4, 250: 2}
    budget = {100: 400000, 150: 400000, 200: 1 << 22, 250: 1 << 22}
    ev = w.random_3sat_sets(per_n=max(per_n.values()), ns=tuple(per_n))
    from concurrent.futures import ProcessPoolExecutor
    cores = min(len(os.sched_getaffinity(0)), 16)
    for n, count in per_n.items():
        cnfs = ev[n][:count]
        raw = ctx.cnf_from_arrays(*w.concat(cnfs))
        tuned, rep = ctx.autotune(raw, sample=min(count, 32), reps=1, max_cubes=400000)
        k = tuned["k"]
        base = dict(k=k, leaves_per_round=tuned["leaves_per_round"], chunk_log2=tuned["chunk_log2"],
                    grid=tuned["grid"], max_cubes=budget[n])
        dv, vd = decide_stats(ctx, raw, count, k=k, max_cubes=budget[n], device_split=True)
        nh = host_n[n]
        raw_h = raw if nh == count else ctx.cnf_from_arrays(*w.concat(cnfs[:nh]))
        st, vs = decide_stats(ctx, raw_h, nh, **base)
        nl = learned_n[n]
        raw_l = raw if nl == count else ctx.cnf_from_arrays(*w.concat(cnfs[:nl]))
        le, vl = decide_stats(ctx, raw_l, nl, **base,
                              learned=mlp_s.scorer(LEARNED_CANDIDATES, LEARNED_RESCORE))
        assert all(a == b or "UNKNOWN" in (a, b) for a, b in zip(vd, vs))
        assert all(a == b or "UNKNOWN" in (a, b) for a, b in zip(vd, vl))
        no = oracle_n[n]
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=min(cores, no)) as ex:
            ov = list(ex.map(_oracle_3sat, cnfs[:no]))
        oracle_s = time.perf_counter() - t0
        # a query left UNKNOWN by either side (budget) is counted, not compared
        agree = [a == b for a, b in zip(ov, vd[:no]) if "UNKNOWN" not in (a, b)]
        assert all(agree), "oracle disagrees on random 3-SAT"
        st_same = decide_stats(ctx, raw_l, nl, **base)[0] if nl != nh else st
        leg = {"instances": count, "of": 2500, "k_autotuned": k, "tuned": tuned,
               "static_device_split": dv, "static_host_split": dict(st, instances=nh),
               "learned_host_split": dict(le, instances=nl),
               "learned_vs_static_host": {"instances": nl,
                                          "leaf_ratio": round(le["leaves"] / max(st_same["leaves"], 1), 3),
                                          "time_ratio": round(le["ms"] / max(st_same["ms"], 1e-9), 3)},
               "device_vs_host_static_ms_per_instance": [round(dv["ms"] / count, 3), round(st["ms"] / nh, 3)],
               "oracle_sample": no, "oracle_seconds": round(oracle_s, 1),
               "oracle_unknown": sum(a == "UNKNOWN" for a in ov),
               "path_unknown_in_sample": sum(b == "UNKNOWN" for b in vd[:no]),
               "oracle_agreement": (sum(agree) / len(agree)) if agree else None}
        out[f"random3sat_n{n}"] = leg
        log(f"3-SAT n={n}: {leg}")
    # partition queries, all 1024
    gens = w.partition_batch()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    labels = [g.label for g in gens]
    st, _ = decide_stats(ctx, cnf, len(gens), labels, k=30, max_cubes=3000)
    le, _ = decide_stats(ctx, cnf, len(gens), labels, k=30, max_cubes=3000,
                         learned=mlp_q.scorer(LEARNED_CANDIDATES, 1))
    wo, _ = decide_stats(ctx, cnf, len(gens), labels, k=30, max_cubes=3000, scorer="word")
    out["partition_1024"] = {"static": st, "learned": le, "word": wo}
    log(f"partition queries: {out['partition_1024']}")
    # lower-bound stencil reads (offset < 0), 256 of them, static cubing
    gens = w.batch_lower()
    t0 = time.perf_counter()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens])
    bbl = 1000.0 * (time.perf_counter() - t0)
    dec = [decide_stats(ctx, cnf, len(gens), [g.label for g in gens], k=30, leaves_per_round=1,
                        chunk_log2=12)[0] for _ in range(3)]
    best = min(dec, key=lambda d: d["ms"])
    out["lower_bound_256"] = {"bitblast_ms": round(bbl, 2), "decide": best,
                              "queries_per_s": round(len(gens) / ((bbl + best["ms"]) / 1000.0), 1)}
    log(f"lower-bound reads: {out['lower_bound_256']}")
    # the same guarded 1-D accesses with 32-bit machine integers
    from paper_2601_21552_amd import _lib
    gens = w.batch_wrap(m=32)
    t0 = time.perf_counter()
    cnf = ctx.bitblast([g.query.arrays()[:2] for g in gens], flags=_lib.BB_WRAP(32))
    bbw = 1000.0 * (time.perf_counter() - t0)
    st, verd = decide_stats(ctx, cnf, len(gens), [g.label for g in gens], k=30, leaves_per_round=1,
                            chunk_log2=12, max_cubes=300)
    out["wrap32_256"] = {"bitblast_ms": round(bbw, 2), "decide": st,
                         "sat_found": sum(v == "SAT" for v, g in zip(verd, gens) if g.label == "SAT"),
                         "sat_labels": sum(g.label == "SAT" for g in gens)}
    log(f"32-bit wrap-around: {out['wrap32_256']}")
    # queries that the front-end emits from 128 small generated programs
    from paper_2601_21552_amd import frontend
    import workloads.program as wp
    progs = wp.random_programs(seed=14, n=128)
    t0 = time.perf_counter()
    aqs = [a for p in progs for a in frontend.analyse(p, lower=True)]
    t1 = time.perf_counter()
    cnf = ctx.bitblast([a.query.arrays()[:2] for a in aqs])
    t2 = time.perf_counter()
    tuned, rep = ctx.autotune(cnf, sample=len(aqs), reps=1)
    dec_t = [decide_stats(ctx, cnf, len(aqs), **tuned)[0] for _ in range(3)]
    best_t = min(dec_t, key=lambda d: d["ms"])
    fe_ms, bbp = 1000.0 * (t1 - t0), 1000.0 * (t2 - t1)
    out["programs_128"] = {"queries": len(aqs), "frontend_ms": round(fe_ms, 2), "bitblast_ms": round(bbp, 2),
                           "tuned": tuned, "decide_tuned": best_t,
                           "queries_per_s": round(len(aqs) / ((fe_ms + bbp + best_t["ms"]) / 1000.0), 1)}
    log(f"programs: {out['programs_128']}")
    # use-after-free live-set analysis (host only) on 64 generated programs
    from paper_2601_21552_amd import uaf
    uprogs = wp.random_uaf_programs(seed=23, n=64)
    t0 = time.perf_counter()
    reports = sum(len(uaf.analyse(p)) for p in uprogs)
    out["uaf_64"] = {"programs": len(uprogs), "reports": reports,
                     "analysis_ms": round(1000.0 * (time.perf_counter() - t0), 2)}
    return out


def secondary_1d(ctx, stream, args, mlp_q):
    """The 1-D batch (256 queries, k = 30) under each ordering: queries/s."""
    import workloads as w
    from paper_2601_21552_amd import api
    gens = w.batch_1d()
    steps = Steps(ctx, api.pack_queries([g.query.arrays()[:2] for g in gens]), gens, stream, args)
    out = {}
    for name, extra in (("static", {}), ("word", dict(scorer="word")),
                        ("learned", dict(learned=mlp_q.scorer(LEARNED_CANDIDATES, LEARNED_RESCORE_ACCESS)))):
        r = steps.run(dict(k=30, leaves_per_round=1, chunk_log2=12, **extra))
        out[name] = {"queries_per_s": round(len(gens) / (r["ms_per_step"] / 1000.0), 1),
                     "ms_per_step": round(r["ms_per_step"], 3), "agree": r["agree"]}
    return out


def leaf_profile(args):
    """Exhaustive leaf evaluation, the leaf kernel's own roof: COUNT mode
    over every leaf of 64 seeded uniform random 3-SAT formulas (n = 64,
    m = 273, the ratio 4.26 of the 3-SAT sets), split on the host to at most
    28 active variables (about 700 leaves, 10 M blocks of 4096 assignments
    per call).  Prints one JSON line: the leaf kernel's word operations
    (64 x (|c| + 1) per evaluated clause-block, two int32 ops each) per
    second against the int32 VALU peak, per leaf-evaluation variant."""
    import numpy as np
    import torch
    from oracle import cnf_ref
    from paper_2601_21552_amd import api
    import workloads as w
    ctx = api.Context(0)
    rng = np.random.Generator(np.random.PCG64(401))
    cnfs = [w.random_ksat(64, 273, 3, rng) for _ in range(64)]
    raw = ctx.cnf_from_arrays(*w.concat(cnfs))
    cubes = ctx.split(raw, k=args.leaf_k)
    out = {"metric": "leaf kernel int32 lane-ops/s (exhaustive COUNT leaves)", "unit": "TOP/s",
           "peak": PEAK_INT32_TOPS, "workload": f"64 random 3-SAT n=64 m=273 seed 401, k={args.leaf_k}",
           "variants": {}}
    # the oracle's exact model counts for a few formulas: the leaves must add up
    check = {qi: cnf_ref.count(cnfs[qi]) for qi in range(4)}
    for name, extra in LEAF_VARIANTS.items():
        if args.leaf_variant and name != args.leaf_variant:
            continue
        opts = dict(mode=1, **extra)
        for _ in range(args.warmup):
            res = ctx.solve(raw, cubes, **opts)
        for qi, want in check.items():
            r = res.result(qi)
            cv = cubes.view(qi)
            got = sum(res.leaf(qi, c)["count"] << res.leaf(qi, c)["m"]
                      for c in range(len(cv["kind"])) if not res.leaf(qi, c)["refuted"])
            assert got == want, (name, qi, got, want)
        torch.cuda.synchronize()
        leaf_ms = launches = 0.0
        word_ops = clause_blocks = blocks = 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = ctx.solve(raw, cubes, **opts)
            tm = res.timing()
            leaf_ms += tm["leaf"]
            launches += tm["leaf_launches"]
            for qi in range(len(cnfs)):
                r = res.result(qi)
                word_ops += r["word_ops"]
                clause_blocks += r["clause_blocks"]
                blocks += r["blocks_evaluated"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        avg = leaf_ms / max(launches, 1)
        ach = 2 * word_ops / launches / (avg * 1e-3) / 1e12
        out["variants"][name] = {
            "avg_launch_ms": round(avg, 4), "launches": launches, "wall_ms_per_call": round(1000 * wall / args.steps, 3),
            "word_ops_per_launch": word_ops / launches, "clause_blocks_per_launch": clause_blocks / launches,
            "blocks_per_launch": blocks / launches, "achieved_tops": round(ach, 4),
            "frac": round(ach / PEAK_INT32_TOPS, 5),
            "clause_block_tops": round(OPS_PER_CLAUSE_BLOCK * clause_blocks / launches / (avg * 1e-3) / 1e12, 4)}
        log(f"leaf variant {name}: {out['variants'][name]}")
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch_2d", choices=sorted(WORKLOADS))
    ap.add_argument("--form", default="auto", choices=("auto", "static", "learned", "word"),
                    help="ordering of the headline value (auto: learned if it agrees 100%%, else static "
                         "if it does, else word)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-form", action="store_true",
                    help="time only the --form ordering (profiling runs)")
    ap.add_argument("--no-gain", action="store_true", help="skip the 3-SAT / partition / other legs")
    ap.add_argument("--no-micro", action="store_true", help="skip the microbenchmark peaks")
    ap.add_argument("--leaf-profile", action="store_true",
                    help="only the exhaustive leaf-evaluation workload (the leaf kernel's roof)")
    ap.add_argument("--leaf-k", type=int, default=28)
    ap.add_argument("--leaf-variant", default="", help="one variant of the leaf profile")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, metavar="PATH",
                    help="autotuner choices to load first (JSON lines keyed by GPU architecture; "
                         "'' or a missing file: tune every batch live)")
    ap.add_argument("--tune-cache-save", default="", metavar="PATH",
                    help="write the context's autotuner choices here at the end")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device 3 times (a plain copy kernel of known "
                         "size, to scale hardware byte counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(queries are independent: a multi-GPU run would shard the batch "
              "with no collective)", file=sys.stderr)
        sys.exit(2)

    if args.leaf_profile:
        leaf_profile(args)
        return

    import torch
    from paper_2601_21552_amd import api

    if args.copy_calibration:
        n = args.copy_calibration << 18          # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    micro = None
    if not args.no_micro:
        from paper_2601_21552_amd import kmicro
        micro = kmicro.measure()
        log(f"microbenchmark peaks: {micro}")

    gens = make_batch(args.workload)
    packed = api.pack_queries([g.query.arrays()[:2] for g in gens])
    ctx = api.Context(0)
    if args.tune_cache and os.path.exists(args.tune_cache):
        log(f"autotuner choices loaded from {os.path.relpath(args.tune_cache, ROOT)}: "
            f"{ctx.tune_cache_load(args.tune_cache)}")
    stream = torch.cuda.current_stream()
    steps = Steps(ctx, packed, gens, stream, args)
    n = len(gens)
    max_cubes = MAX_CUBES[args.workload]

    import workloads as w
    names = [args.form] if (args.only_form and args.form != "auto") else ["static", "word", "learned"]
    # the learned scorer, trained on traces of other seeds' access batches
    # (when a leg uses it)
    mlp_q, scorer_info = None, None
    if "learned" in names or not args.only_form:
        t0 = time.perf_counter()
        tr = [ctx.bitblast([g.query.arrays()[:2] for g in w.batch_1d(seed=102)]),
              ctx.bitblast([g.query.arrays()[:2] for g in w.batch_2d(seed=103, n=1024)])]
        mlp_q, scorer_info = train_scorer(ctx, tr, k=30, epochs=4, seed=2)
        scorer_info["seconds"] = round(time.perf_counter() - t0, 1)
        log(f"access-query scorer trained: {scorer_info}")

    # per ordering: autotuned options (static / word; the learned form runs
    # at the word ordering's point, since on access queries it also walks
    # input words by their top bits), timed steps, agreement with the labels
    cnf0 = ctx.bitblast_packed(*packed)
    forms, runs = {}, {}
    tuned = {}
    for name in names:
        t0 = time.perf_counter()
        if name in ("static", "word"):
            tuned[name], rep = ctx.autotune(cnf0, sample=128, reps=1, scorer=name, graph=True,
                                            max_cubes=max_cubes)
        else:
            if "word" not in tuned:
                tuned["word"], rep = ctx.autotune(cnf0, sample=128, reps=1, scorer="word", graph=True,
                                                  max_cubes=max_cubes)
            rep = {"points": 0}
        tune_s = time.perf_counter() - t0
        opts = dict(tuned["word" if name == "learned" else name], max_cubes=max_cubes)
        if name == "learned":
            opts.pop("scorer", None)
            opts["learned"] = mlp_q.scorer(LEARNED_CANDIDATES, LEARNED_RESCORE_ACCESS)
        # a form below 100% agreement cannot give the headline: one timed call
        r = steps.run(opts, steps=1, warmup=1)
        timed_steps = 1
        if r["agree"] == 1.0 and r["unknown"] == 0:
            r = steps.run(opts)
            timed_steps = args.steps
        runs[name] = (r, opts)
        forms[name] = {"queries_per_s": round(n / (r["ms_per_step"] / 1000.0), 3),
                       "ms_per_step": round(r["ms_per_step"], 3), "agree": r["agree"], "unknown": r["unknown"],
                       "first_call_ms": round(r["first_ms"], 2), "bitblast_ms": round(r["bitblast_ms"], 3),
                       "tune_s": round(tune_s, 2), "tune_points": rep["points"], "timed_steps": timed_steps,
                       "options": {k: v for k, v in opts.items() if k != "learned"}}
        log(f"form {name}: {forms[name]}")
    if args.form == "auto":
        head = next((f for f in ("learned", "static", "word") if f in forms and forms[f]["agree"] == 1.0),
                    max(forms, key=lambda f: forms[f]["agree"]))
    else:
        head = args.form
    run, opts = runs[head]

    # per-kernel events: the same steps eagerly (graph replays carry no
    # per-dispatch events), HIP events bracketing each dispatch
    ev_opts = dict(opts, graph=False)
    ev = steps.run(ev_opts, warmup=1)
    tkey = traffic_key(args.workload, {k: v for k, v in ev_opts.items() if k != "learned"} | {"form": head})
    roofline, detail = kernel_accounting(steps, ev, tkey)
    if micro:
        for line in (roofline, roofline["other"]):
            mp = micro["valu_int32_tops"] if line["bound"] == "alu" else micro["hbm_gbs"]
            line["measured_peak"] = mp
            line["frac_of_measured_peak"] = round(line["achieved"] / mp, 5) if mp else None
    detail["eager_ms_per_step"] = round(ev["ms_per_step"], 3)
    detail["bitblast_ms_per_step"] = round(run["bitblast_ms"], 3)
    detail["first_call_ms"] = round(run["first_ms"], 2)
    detail["traffic_key"] = tkey

    secondary = None
    gain = None
    if not args.only_form:
        secondary = {"batch_1d_256": secondary_1d(ctx, stream, args, mlp_q)}
        log(f"1-D batch: {secondary}")
        if not args.no_gain:
            tr3 = w.random_3sat_train(per_n=48)
            tb = [ctx.cnf_from_arrays(*w.concat(tr3[100])), ctx.cnf_from_arrays(*w.concat(tr3[150][:16]))]
            mlp_s = train_scorer(ctx, tb, k=16, epochs=6, seed=4, candidates=16, depth=40)
            gain = gain_legs(ctx, mlp_q, mlp_s, args)

    cpu = None
    if not args.no_cpu_baseline:
        res_last = run["results"][-1]
        cpu = cpu_baseline_leg(gens, run["cnf"], res_last.verdicts(), res_last)
        log(f"cpu baseline: {cpu}")
        assert cpu["oracle_agreement"] == 1.0 or cpu["oracle_unknown"] > 0

    out = {
        "metric": "OOB queries decided/sec at 100% oracle agreement, learned vs static cubing",
        "value": forms[head]["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": forms[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": WORKLOADS[args.workload], "queries": n, "scorer": head,
                   "options": forms[head]["options"], "max_cubes": max_cubes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "micro_peaks": micro,
        "learned_scorer": scorer_info,
        "secondary": secondary,
        "gain": gain,
        "detail": detail,
    }
    if args.tune_cache_save:
        ctx.tune_cache_save(args.tune_cache_save)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
