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

WORKLOADS = {
    2: ("config2: 256 seeded 1-D OOB queries, widths 8-16 bits, s in {1,2,4,8}, "
        "c in 0..16, 128 guarded (UNSAT) / 64 unguarded + 64 off-by-one (SAT); "
        "static cubing k=30"),
    1: "config1: one 12-bit guarded idx<N query (UNSAT), static cubing k=30",
}


def make_batch(config: int):
    import workloads as w
    if config == 1:
        return [w.config1("lt")]
    return w.config2()


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--k", type=int, default=30)
    ap.add_argument("--leaves-per-round", type=int, default=4)
    ap.add_argument("--chunk-log2", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(queries are independent: a multi-GPU run would shard the batch "
              "with no collective)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_21552_amd import api

    gens = make_batch(args.config)
    arrays = [g.query.arrays()[:2] for g in gens]
    labels = [g.label for g in gens]
    ctx = api.Context(0)
    stream = torch.cuda.current_stream()
    opts = dict(k=args.k, leaves_per_round=args.leaves_per_round, chunk_log2=args.chunk_log2)

    def step():
        cnf = ctx.bitblast(arrays)
        res = ctx.decide(cnf, stream=stream, **opts)
        return cnf, res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps

    # agreement and accounting over the timed steps
    from oracle import query_ref
    n_root = n_dev = n_unknown = 0
    clause_blocks = 0
    leaf_ms = up_ms = 0.0
    leaf_launches = up_launches = 0
    split_ms = verify_ms = 0.0
    for cnf, res in results:
        for i, g in enumerate(gens):
            r = res.result(i)
            assert r["verdict"] == labels[i], (g.query.name, r)
            if r["verdict"] == "SAT":
                assert r["witness_checked"]
        tm = res.timing()
        leaf_ms += tm["leaf"]
        up_ms += tm["up"]
        leaf_launches += int(tm["leaf_launches"])
        up_launches += int(tm["up_launches"])
        split_ms += tm["split"]
        verify_ms += tm["verify"]
    cnf, res = results[-1]
    for i, g in enumerate(gens):
        r = res.result(i)
        n_root += r["how"] == "root"
        n_dev += r["how"] == "device"
        n_unknown += r["verdict"] == "UNKNOWN"
        clause_blocks += r["clause_blocks"]
        if r["verdict"] == "SAT":
            assert query_ref.int_eval(g.query, res.witness(i, g.query.n_vars))

    steps = args.steps
    leaf_avg_ms = leaf_ms / max(leaf_launches, 1)
    ops_per_step = OPS_PER_CLAUSE_BLOCK * clause_blocks
    leaf_launches_per_step = leaf_launches / steps
    achieved = (ops_per_step / max(leaf_launches_per_step, 1)) / (leaf_avg_ms * 1e-3) / 1e12 \
        if leaf_ms > 0 else 0.0
    roofline = {"bound": "alu", "kernel": "leaf_kernel", "achieved": round(achieved, 4),
                "peak": PEAK_INT32_TOPS, "unit": "TOP/s (int32 VALU lane-ops)",
                "frac": round(achieved / PEAK_INT32_TOPS, 5), "traffic": None,
                "avg_launch_ms": round(leaf_avg_ms, 4),
                "launches_per_step": leaf_launches_per_step,
                "clause_blocks_per_step": clause_blocks,
                "up_kernel_avg_launch_ms": round(up_ms / max(up_launches, 1), 4)}

    cpu = None
    agree = None
    if not args.no_cpu_baseline:
        cores = len(os.sched_getaffinity(0))
        cores = min(cores, 16)
        v, overd, dt = oracle_leg(gens, cores)
        agree = sum(a == b for a, b in zip(overd, labels)) / len(labels)
        assert agree == 1.0, "oracle disagrees with the path"
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
        "config": {"workload": WORKLOADS[args.config], "queries": len(gens), "k": args.k,
                   "scorer": "static", "leaves_per_round": args.leaves_per_round,
                   "chunk_log2": args.chunk_log2},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"decided_at_root": n_root, "decided_on_device": n_dev,
                   "unknown": n_unknown, "oracle_agreement": agree,
                   "host_split_ms_per_step": round(split_ms / steps, 3),
                   "verify_ms_per_step": round(verify_ms / steps, 3),
                   "leaf_kernel_ms_per_step": round(leaf_ms / steps, 3),
                   "up_kernel_ms_per_step": round(up_ms / steps, 3)},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
