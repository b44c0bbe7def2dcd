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


def kernel_source_digest() -> str:
    """Digest of the rating kernels' sources; HBM traffic measured for
    another version of them is not reported."""
    import hashlib

    h = hashlib.sha256()
    for f in ("common.h", "lp_kernels.hip"):
        h.update(open(os.path.join(ROOT, "paper_1402_3281_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` from profiles/traffic.json (rocprofv3
    FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_digest") != kernel_source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def copy_calibration(mbytes: int) -> int:
    """Plain device copy of a known size (for scaling rocprofv3 counters)."""
    import torch

    n = mbytes * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "dispatches": 3}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scale", type=int, default=22, help="R-MAT scale (log2 of the node count of both graphs)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calib_copy_mb:
        return copy_calibration(args.calib_copy_mb)
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
    ms_per_step = elapsed * 1000.0 / args.steps
    value = visits / elapsed

    # one more step, untimed, with HIP events around every rating launch
    ctx.profile(True)
    step()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)

    # roofline of the dominant rating kernel: algorithmic bytes per launch
    # (4 B neighbour id + 4 B neighbour label [+ 4 B edge weight] per edge
    # visit, 32 B per rated node) / mean launch duration (HIP events)
    names = ["k_rate_small (degree 1-128)", "k_rate_mid (degree 129-1024)", "k_rate_large (degree 1025-4096)",
             "hub path (4 kernels, degree > 4096)"]
    launches = max(prof["kernel_launches"], 1)
    dom = max(range(3), key=lambda b: prof["kernels"][b]["ms"])
    kd = prof["kernels"][dom]
    avg_ms = kd["ms"] / launches
    bytes_per_launch = kd["bytes"] / launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    step_kernels = [{"kernel": names[b], "ms_per_round": prof["kernels"][b]["ms"] / launches,
                     "GBps": (prof["kernels"][b]["bytes"] / (prof["kernels"][b]["ms"] * 1e-3) / 1e9)
                     if prof["kernels"][b]["ms"] > 0 else 0.0} for b in range(4)]

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t1 = time.perf_counter()
        cv = 0
        rounds = 0
        for g in graphs:
            og = oracle.OGraph.of(g)
            _, _, U = oracle.bounds(g.n, 1, k, 3, 100, 14)
            r = oracle.cluster(og, U, 10, 1, 1)
            cv += r.visits
            rounds += r.rounds
        ct = time.perf_counter() - t1
        cpu = {"value": cv / ct, "unit": "edge visits/s", "cores": 1, "kind": "oracle",
               "sample": "oracle level-0 clustering (up to 10 LP rounds with the coarsening stop rule) of both "
                         f"graphs, single thread, gcc -O2: {rounds} rounds, {cv} visits in {ct:.1f}s"}

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
        "visits_per_step": visits // max(args.steps, 1),
        "rating_kernels": step_kernels,
        "roofline": {
            "bound": "hbm",
            "kernel": names[dom],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_for(names[dom]),
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
