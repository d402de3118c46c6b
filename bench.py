"""Throughput of the OOB-query decision path on one MI355X.

One step = the whole path for one batch: query DAGs -> normalisation and
Tseitin CNF (host) -> lazy cube splitting (host) -> device unit propagation
and bit-sliced leaf evaluation (gfx950) -> verified verdicts and witnesses.
Default workload: 256 seeded 1-D access queries (widths 8-16 bits, element
size s in {1,2,4,8}, header c in 0..16; 128 with the correct guard, 128
unguarded or off by one), static cubing with k = 30.

Prints one JSON line: queries decided per second over the timed steps, the
roofline of the dominant kernel (HIP events on the library's stream) and the
CPU oracle timed on this host's cores.  Every step's verdicts must agree with
the oracle (and the generators' labels); witnesses are re-checked exactly.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 39.3216   # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz (int32 VALU)
PEAK_HBM_GBS = 8000.0
# per evaluated clause-block (one residual clause against 4096 assignments):
# the 64-bit AND of the clause's satisfaction word into each of the 64 lanes'
# accumulators = 64 lanes x 2 int32 ops
OPS_PER_CLAUSE_BLOCK = 128

# HBM bytes per launch from two rocprofv3 counter passes over this bench's
# default workload (FETCH_SIZE / 0.5 + WRITE_SIZE, both scaled by what they
# read for a device copy of known size), valid only for the kernel source
# they were taken on
MEASURED_TRAFFIC = {
    "device_hip_sha256_16": "dffad7f9ea90893e",
    "up_kernel": 14_491_136,
    "leaf_kernel": 3_004_501,
}

# learned ordering: candidates scored per decision node, and the levels
# below a scored node that reuse its ranking (fewer device scoring passes).
# The access queries are shallow trees (about 27 decisions to a k = 30
# leaf): one ranking per 32 levels serves them.  With the scorer trained here
# (seeded), 16 and 64 levels pick leaves whose first model lies deep in the
# enumeration (3 ms of leaf kernel per step against 0.4 ms).  The random
# 3-SAT trees are deeper and are rescored every 4 levels.
LEARNED_CANDIDATES = 16
LEARNED_RESCORE = 4
LEARNED_RESCORE_ACCESS = 32

WORKLOADS = {
    "batch_1d": ("256 seeded 1-D OOB queries, widths 8-16 bits, s in {1,2,4,8}, "
                 "c in 0..16, 128 guarded (UNSAT) / 64 unguarded + 64 off-by-one (SAT); "
                 "static cubing k=30"),
    "single": "one 12-bit guarded idx<N query (UNSAT), static cubing k=30",
}


def make_batch(workload: str):
    import workloads as w
    if workload == "single":
        return [w.single_access("lt")]
    return w.batch_1d()


def oracle_leg(gens, cores: int):
    """The oracle as it stands, timed on this host; returns (value, verdicts,
    seconds, cores)."""
    from concurrent.futures import ProcessPoolExecutor
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        verdicts = list(ex.map(_oracle_one, [g.query for g in gens], chunksize=4))
    dt = time.perf_counter() - t0
    return len(gens) / dt, verdicts, dt


def _oracle_one(q):
    from oracle import query_ref
    return query_ref.decide(q)[0]


def measured_traffic(args):
    """The counter figures when they apply: same kernel source, default
    workload and launch options; else None."""
    import hashlib
    src = os.path.join(ROOT, "paper_2601_21552_amd", "csrc", "device.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    default = (args.workload == "batch_1d" and args.k == 30 and args.leaves_per_round == 1
               and args.chunk_log2 == 12)
    if sha != MEASURED_TRAFFIC["device_hip_sha256_16"] or not default:
        return None
    return MEASURED_TRAFFIC


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


def gain_legs(ctx, mlp_q, log):
    """Learned vs static on samples of the random 3-SAT workload (scorer
    trained on disjoint-seed instances) and the partition queries (scorer
    trained on 1-D / 2-D access traces): verdicts must agree; leaves, cubes
    and wall time are reported."""
    import workloads as w
    out = {}
    # random 3-SAT: n = 100 and 150, k = 16
    tr = w.random_3sat_train(per_n=48)
    tr_batches = [ctx.cnf_from_arrays(*w.concat(tr[100])),
                  ctx.cnf_from_arrays(*w.concat(tr[150][:16]))]
    mlp_s, info = train_scorer(ctx, tr_batches, k=16, epochs=6, seed=4, candidates=16, depth=40)
    log(f"3-SAT scorer trained: {info}")
    ev = w.random_3sat_sets(per_n=128, ns=(100, 150))
    for n, count in ((100, 128), (150, 32)):
        cnfs = ev[n][:count]
        raw = ctx.cnf_from_arrays(*w.concat(cnfs))
        st, vs = decide_stats(ctx, raw, count, k=16, max_cubes=400000)
        le, vl = decide_stats(ctx, raw, count, k=16, max_cubes=400000,
                              learned=mlp_s.scorer(LEARNED_CANDIDATES, LEARNED_RESCORE))
        assert all(a == b or "UNKNOWN" in (a, b) for a, b in zip(vs, vl))
        leg = {"instances": count, "static": st, "learned": le,
               "leaf_ratio": round(le["leaves"] / max(st["leaves"], 1), 3),
               "time_ratio": round(le["ms"] / max(st["ms"], 1e-9), 3)}
        if n == 100:
            # checked against the oracle in the CPU-baseline leg
            out["_random3sat_n100_check"] = (cnfs, vs)
        out[f"random3sat_n{n}"] = leg
        log(f"3-SAT n={n}: {leg}")
    out["random3sat_scorer"] = info
    # 4096 2-D accesses of uneven width in one decide call, autotuned and
    # captured as HIP graphs (word ordering)
    gens3 = w.batch_2d()
    t0 = time.perf_counter()
    cnf3 = ctx.bitblast([g.query.arrays()[:2] for g in gens3])
    bb3 = 1000.0 * (time.perf_counter() - t0)
    tuned, rep = ctx.autotune(cnf3, sample=128, reps=1, scorer="word", graph=True)
    labels3 = [g.label for g in gens3]
    dec = [decide_stats(ctx, cnf3, len(gens3), labels3, max_cubes=20000, **tuned)[0] for _ in range(2)]
    best = min(dec, key=lambda d: d["ms"])
    out["batch_4096_2d"] = {"bitblast_ms": round(bb3, 1), "tuned": tuned,
                            "tune_points": rep["points"], "decide": best,
                            "queries_per_s": round(len(gens3) / ((bb3 + best["ms"]) / 1000.0), 1)}
    log(f"4096 2-D accesses: {out['batch_4096_2d']}")
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
    # the same guarded 1-D accesses with 32-bit machine integers: byte sizes
    # that wrap are found SAT; the wrap-safe UNSAT ones may stay UNKNOWN
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
    # (host and kernel analysis, upper and lower bound of every access)
    from paper_2601_21552_amd import frontend
    import workloads.program as wp
    progs = wp.random_programs(seed=14, n=128)
    t0 = time.perf_counter()
    aqs = [a for p in progs for a in frontend.analyse(p, lower=True)]
    t1 = time.perf_counter()
    cnf = ctx.bitblast([a.query.arrays()[:2] for a in aqs])
    t2 = time.perf_counter()
    dec = [decide_stats(ctx, cnf, len(aqs), k=30, leaves_per_round=1, chunk_log2=12)[0]
           for _ in range(3)]
    best = min(dec, key=lambda d: d["ms"])
    # the UNSAT queries that the root stage leaves open end in exhaustive
    # leaves of up to 2^30 assignments at k = 30; the tuner trades leaf size
    # for splitting
    tuned, rep = ctx.autotune(cnf, sample=len(aqs), reps=1)
    dec_t = [decide_stats(ctx, cnf, len(aqs), **tuned)[0] for _ in range(3)]
    best_t = min(dec_t, key=lambda d: d["ms"])
    fe_ms, bbp = 1000.0 * (t1 - t0), 1000.0 * (t2 - t1)
    out["programs_128"] = {"queries": len(aqs), "frontend_ms": round(fe_ms, 2),
                           "bitblast_ms": round(bbp, 2), "decide_k30": best,
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
    log(f"use after free: {out['uaf_64']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch_1d", choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=30)
    ap.add_argument("--leaves-per-round", type=int, default=1)
    ap.add_argument("--chunk-log2", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the word / learned forms")
    ap.add_argument("--no-gain", action="store_true", help="skip the learned-vs-static legs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device 3 times (a plain copy kernel of known "
                         "size, to scale hardware byte counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(queries are independent: a multi-GPU run would shard the batch "
              "with no collective)", file=sys.stderr)
        sys.exit(2)

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

    gens = make_batch(args.workload)
    arrays = [g.query.arrays()[:2] for g in gens]
    # the batch in the boundary's input layout (all node records and roots
    # with per-query offsets), as a caller holding the query DAGs has it
    packed = api.pack_queries(arrays)
    labels = [g.label for g in gens]
    ctx = api.Context(0)
    stream = torch.cuda.current_stream()
    opts = dict(k=args.k, leaves_per_round=args.leaves_per_round, chunk_log2=args.chunk_log2)

    bb_ms = []

    def run_steps(extra):
        def step():
            t0 = time.perf_counter()
            cnf = ctx.bitblast_packed(*packed)
            bb_ms.append(1000.0 * (time.perf_counter() - t0))
            res = ctx.decide(cnf, stream=stream, **opts, **extra)
            return cnf, res

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        last_cnf = None
        for _ in range(args.steps):
            cnf, res = step()
            out.append(res)
            # a step's CNF is released when the next step replaces it, as in a
            # pipeline that frees each batch after deciding it; the results stay
            last_cnf = cnf
            del cnf
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        for res in out:
            for i, g in enumerate(gens):
                r = res.result(i)
                assert r["verdict"] == labels[i], (g.query.name, r, extra)
                if r["verdict"] == "SAT":
                    assert r["witness_checked"]
        return 1000.0 * elapsed / args.steps, out, last_cnf

    ms_per_step, results, last_cnf = run_steps({})
    bitblast_ms = sorted(bb_ms[args.warmup:])[len(bb_ms[args.warmup:]) // 2]

    # accounting over the timed steps (every SAT witness was checked by the
    # library's own verifier; the oracle's checks run in the CPU-baseline leg)
    n_root = n_dev = n_unknown = 0
    clause_blocks = leaves_sent = leaves_refuted = blocks_evaluated = 0
    leaf_ms = up_ms = 0.0
    leaf_launches = up_launches = 0
    split_ms = verify_ms = 0.0
    for res in results:
        tm = res.timing()
        leaf_ms += tm["leaf"]
        up_ms += tm["up"]
        leaf_launches += int(tm["leaf_launches"])
        up_launches += int(tm["up_launches"])
        split_ms += tm["split"]
        verify_ms += tm["verify"]
    cnf, res = last_cnf, results[-1]
    for i, g in enumerate(gens):
        r = res.result(i)
        n_root += r["how"] == "root"
        n_dev += r["how"] == "device"
        n_unknown += r["verdict"] == "UNKNOWN"
        clause_blocks += r["clause_blocks"]
        leaves_sent += r["leaves_sent"]
        leaves_refuted += r["leaves_refuted"]
        blocks_evaluated += r["blocks_evaluated"]

    steps = args.steps
    # algorithmic work of the last step (every step does the same work)
    up_bytes = 0
    for i in range(len(gens)):
        r = res.result(i)
        if r["leaves_sent"]:
            v = cnf.view(i)
            up_bytes += r["leaves_sent"] * 4 * (v["n_clauses"] + 1 + len(v["lits"]))
    leaf_avg_ms = leaf_ms / max(leaf_launches, 1)
    up_avg_ms = up_ms / max(up_launches, 1)
    kernels = {
        "leaf_kernel": dict(bound="alu", ms_step=leaf_ms / steps, avg=leaf_avg_ms,
                            per_launch=OPS_PER_CLAUSE_BLOCK * clause_blocks / max(leaf_launches / steps, 1),
                            peak=PEAK_INT32_TOPS, unit="TOP/s (int32 VALU lane-ops)", scale=1e12,
                            launches=leaf_launches / steps),
        "up_kernel": dict(bound="hbm", ms_step=up_ms / steps, avg=up_avg_ms,
                          per_launch=up_bytes / max(up_launches / steps, 1),
                          peak=PEAK_HBM_GBS, unit="GB/s (CNF bytes per cube)", scale=1e9,
                          launches=up_launches / steps),
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms_step"])
    kd = kernels[dom]
    achieved = kd["per_launch"] / (kd["avg"] * 1e-3) / kd["scale"] if kd["avg"] > 0 else 0.0
    traffic = measured_traffic(args)
    roofline = {"bound": kd["bound"], "kernel": dom, "achieved": round(achieved, 4),
                "peak": kd["peak"], "unit": kd["unit"], "frac": round(achieved / kd["peak"], 5),
                "traffic": traffic.get(dom) if traffic else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_launch_ms": round(kd["avg"], 4),
                "launches_per_step": kd["launches"]}
    other = "leaf_kernel" if dom == "up_kernel" else "up_kernel"
    ko = kernels[other]
    oach = ko["per_launch"] / (ko["avg"] * 1e-3) / ko["scale"] if ko["avg"] > 0 else 0.0
    roofline["other"] = {"kernel": other, "bound": ko["bound"], "achieved": round(oach, 4),
                         "traffic": traffic.get(other) if traffic else None,
                         "peak": ko["peak"], "unit": ko["unit"], "frac": round(oach / ko["peak"], 5),
                         "avg_launch_ms": round(ko["avg"], 4), "launches_per_step": ko["launches"]}
    roofline["clause_blocks_per_step"] = clause_blocks
    roofline["up_cnf_bytes_per_step"] = up_bytes

    # the other orderings on the same batch and steps, and the learned
    # scorer's gains on the random 3-SAT and partition workloads
    def log(m):
        print(m, file=sys.stderr, flush=True)

    forms = {"static": round(len(gens) / (ms_per_step / 1000.0), 3)}
    gain = None
    scorer_info = None
    if not (args.no_forms and args.no_gain):
        import workloads as w
        tr = [ctx.bitblast([g.query.arrays()[:2] for g in w.batch_1d(seed=102)]),
              ctx.bitblast([g.query.arrays()[:2] for g in w.batch_2d(seed=103, n=1024)])]
        mlp_q, scorer_info = train_scorer(ctx, tr, k=30, epochs=4, seed=2)
        log(f"access-query scorer trained: {scorer_info}")
    if not args.no_forms:
        for name, extra in (("word", dict(scorer="word")),
                            ("learned", dict(learned=mlp_q.scorer(LEARNED_CANDIDATES, LEARNED_RESCORE_ACCESS)))):
            ms, _, _ = run_steps(extra)
            forms[name] = round(len(gens) / (ms / 1000.0), 3)
        log(f"forms (queries/s): {forms}")
    if not args.no_gain:
        gain = gain_legs(ctx, mlp_q, log)

    cpu = None
    agree = None
    check = gain.pop("_random3sat_n100_check", None) if gain else None
    if not args.no_cpu_baseline:
        # the CPU-baseline leg: the oracle timed on this host, and its checks
        # of the path's verdicts and witnesses
        from oracle import cnf_ref, query_ref
        cores = len(os.sched_getaffinity(0))
        cores = min(cores, 16)
        v, overd, dt = oracle_leg(gens, cores)
        agree = sum(a == b for a, b in zip(overd, labels)) / len(labels)
        assert agree == 1.0, "oracle disagrees with the path"
        res = results[-1]
        for i, g in enumerate(gens):
            if res.result(i)["verdict"] == "SAT":
                assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))
        if check is not None:
            cnfs3, vs3 = check
            ov = [cnf_ref.solve(f)[0] for f in cnfs3]
            gain["random3sat_n100"]["oracle_agreement"] = sum(a == b for a, b in zip(ov, vs3)) / len(vs3)
            assert gain["random3sat_n100"]["oracle_agreement"] == 1.0
        cpu = {"value": round(v, 3), "unit": "queries/s", "cores": cores, "kind": "oracle",
               "sample": f"the full {len(gens)}-query batch once ({dt:.2f} s wall on "
                         f"{cores} processes): root check + own Tseitin + C DPLL per query"}

    out = {
        "metric": "OOB queries decided/sec at 100% oracle agreement, learned vs static cubing",
        "value": round(len(gens) / (ms_per_step / 1000.0), 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": WORKLOADS[args.workload], "queries": len(gens), "k": args.k,
                   "scorer": "static", "leaves_per_round": args.leaves_per_round,
                   "chunk_log2": args.chunk_log2},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "learned_scorer": scorer_info,
        "gain": gain,
        "detail": {"decided_at_root": n_root, "decided_on_device": n_dev,
                   "unknown": n_unknown, "oracle_agreement": agree,
                   "leaves_sent": leaves_sent, "leaves_refuted": leaves_refuted,
                   "blocks_evaluated": blocks_evaluated,
                   "bitblast_ms_per_step": round(bitblast_ms, 3),
                   "host_split_ms_per_step": round(split_ms / steps, 3),
                   "verify_ms_per_step": round(verify_ms / steps, 3),
                   "leaf_kernel_ms_per_step": round(leaf_ms / steps, 3),
                   "up_kernel_ms_per_step": round(up_ms / steps, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
