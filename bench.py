"""Benchmark: SCLaP edge visits/s of the full multilevel partitioner on one
MI355X, with the rating step's HBM roofline fraction and the CPU oracle as a
reported baseline.

Workload (one step): partition an R-MAT graph (scale 22, edge factor 16,
a/b/c/d = .57/.19/.19/.05, 4.19M nodes) and a 2D random geometric graph
(2^22 nodes, average degree 10) into k = 16 blocks, eps = 3/100, f = 14,
coarsening to <= 5000 k = 80,000 nodes, 10 LP rounds per level, LP
refinement on every level.  Inputs are generated on the host, copied to the
device before timing, and stay resident.

value = edge visits (clustering + refinement rounds, both graphs) per
second of the whole step (contraction, initial partition and projection
included).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=int, default=22, help="R-MAT scale (log2 of the node count of both graphs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the partitioner's multi-GPU path is "
              "not built; see the sharding notes in DESIGN.md.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import graphgen
    import paper_1402_3281_amd as sc

    k, thr, scale = 16, 80000, args.scale
    t0 = time.time()
    graphs = [graphgen.rmat(scale, 16, seed=1), graphgen.rgg(1 << scale, 10.0, seed=1)]
    log(f"generated inputs in {time.time() - t0:.1f}s: " + ", ".join(f"{g.name} n={g.n} m={g.m}" for g in graphs))
    torch.cuda.set_device(0)
    devs = [sc.DeviceGraph.from_host(g, rows_sorted=True) for g in graphs]
    parts = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
    ctx = sc.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        out = []
        for d, p in zip(devs, parts):
            _, st = sc.partition(ctx, d, k, threshold=thr, stream=stream, part_out=p)
            out.append(st)
        return out

    for i in range(args.warmup):
        sts = step()
        log(f"warmup {i}: cuts {[s['cut'] for s in sts]} levels {[s['n_level'] for s in sts]}")
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    visits = 0
    visits_c = 0
    sts = []
    for i in range(args.steps):
        sts = step()
        visits += sum(sum(s["visits_c"]) + sum(s["visits_r"]) for s in sts)
        visits_c += sum(sum(s["visits_c"]) for s in sts)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_per_step = elapsed * 1000.0 / args.steps
    value = visits / elapsed

    # roofline of the dominant rating kernel: algorithmic bytes per launch
    # (4 B neighbour id + 4 B neighbour label [+ 4 B edge weight] per edge
    # visit, 32 B per rated node) / mean launch duration (HIP events)
    names = ["k_rate_group<8>", "k_rate_group<16>", "k_rate_group<32>", "k_rate_group<64>", "k_rate_wave<256>",
             "k_rate_wave<1024>", "k_rate_block<2048, 256>", "k_rate_block<8192, 512>", "hub path (4 kernels)"]
    launches = max(prof["kernel_launches"], 1)
    dom = max(range(8), key=lambda b: prof["kernels"][b]["ms"])
    kd = prof["kernels"][dom]
    avg_ms = kd["ms"] / launches
    bytes_per_launch = kd["bytes"] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    step_kernels = [{"kernel": names[b], "ms_per_round": prof["kernels"][b]["ms"] / launches,
                     "GBps": (prof["kernels"][b]["bytes"] / (prof["kernels"][b]["ms"] * 1e-3) / 1e9)
                     if prof["kernels"][b]["ms"] > 0 else 0.0} for b in range(9)]

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t1 = time.perf_counter()
        cv = 0
        for g in graphs:
            og = oracle.OGraph.of(g)
            r = oracle.cluster(og, 19286 if scale == 22 else max(1, int(1.03 * (g.n // k)) // 14), 2, 0, 1)
            cv += r.visits
        ct = time.perf_counter() - t1
        cpu = {"value": cv / ct, "unit": "edge visits/s", "cores": 1, "kind": "oracle",
               "sample": "oracle clustering rounds 1-2 on level 0 of both graphs (single thread, gcc -O2); "
                         f"{cv} visits in {ct:.1f}s"}

    line = {
        "metric": "SCLaP edge visits/s (multilevel partition, clustering + refinement rounds)",
        "value": value,
        "unit": "edge visits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"rmat-s{scale}-ef16 + rgg-2^{scale}-d10, k=16, eps=3/100, f=14, coarsen to <= {thr}, "
                        "10 LP rounds per level, LP refinement on every level",
            "k": k,
            "graphs": [{"name": g.name, "n": g.n, "m": g.m} for g in graphs],
            "cuts": [s["cut"] for s in sts],
            "levels": [s["n_level"] for s in sts],
        },
        "sclap_round_visits_per_s": (prof["visits"] / (prof["round_ms"] * 1e-3)) if prof["round_ms"] > 0 else None,
        "rating_kernels": step_kernels,
        "roofline": {
            "bound": "hbm",
            "kernel": names[dom],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_ms,
            "launches": launches,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
