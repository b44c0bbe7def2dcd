"""Benchmark of the SCLaP multilevel partitioner on one MI355X.

Default workload (`--workload large`, one step): partition an R-MAT graph of
scale 26 (edge factor 16, a/b/c/d = .57/.19/.19/.05, 67.1M nodes, 2.1G
directed entries after symmetrisation and de-duplication) into k = 32 blocks,
eps = 3/100, f = 14, coarsening to at most max(60k, n/(60k)) nodes, 10 LP
rounds per level, LP refinement on every level.  The input is generated on the
host, copied to the device before timing, and stays resident.  value = edge
visits (clustering + refinement rounds) per second of the whole step
(contraction, initial partition and projection included).  The returned blocks
are checked on the host (cut and block weights recomputed, every block within
L_max).  The JSON line carries the HBM roofline of the dominant rating kernel
group and the CPU oracle as a reported baseline.

Other workloads (`--workload`):
  two-graphs  R-MAT scale 22 and a 2D random geometric graph of 2^22 nodes
              (average degree 10), k = 16, coarsening to <= 5000 k nodes.
  batch       512 mixed graphs, batched (every step fused over all graphs)
              versus plain (one graph after the other); graphs/s.
  serve       served Poisson stream of partition jobs under an HBM budget
              versus plain; p50/p99 latency and jobs/s.
  extensions  the Section 4 extensions (V-cycles, sub-rounds, ensembles,
              extra coarse imbalance) on the scale-22 graphs: time, edge
              visits/s and cut per configuration.
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
RATE_KERNELS = ["k_rate_tiny + k_rate_b32 (degree 1-32)", "k_rate_small (bins 3-4, degree 33-128 by default)",
                "k_rate_mid (bins 5-6, degree 129-1024 by default)", "k_rate_large (bin 7, degree up to 4096)",
                "hub path (degree > 4096)", "k_mark + k_mark_big (refinement marking)"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def host_info() -> dict:
    """The host the CPU baseline ran on: logical CPUs and model name."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def kernel_source_digest() -> str:
    """Digest of the rating kernels' sources; HBM traffic measured for
    another version of them is not reported."""
    import hashlib

    h = hashlib.sha256()
    for f in ("common.h", "lp_kernels.hip"):
        h.update(open(os.path.join(ROOT, "paper_1402_3281_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from profiles/traffic.json
    (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    or None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_digest") != kernel_source_digest() or t.get("workload") != workload:
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


def roofline(prof: dict, workload: str) -> tuple[dict, list]:
    """Roofline of the dominant launch group (the one with the most device
    time over the step, among the five rating groups and the refinement
    marking kernels): algorithmic bytes per launch / mean launch duration from
    HIP events.  Rating: 4 B neighbour id + 4 B neighbour label [+ 4 B edge
    weight] per edge visit, no label bytes in a level's first clustering
    round, whose labels are the ids; 32 B per rated node.  Marking: 8 B per
    rated position, 20 B per mover, 5 B per entry of a mover's row plus 16 B
    [+ 4 B edge weight] in rounds that update the block connections.  A
    launch is a round in which the group's kernels ran."""
    groups = range(len(prof["kernels"]))
    dom = max(groups, key=lambda b: prof["kernels"][b]["ms"])
    kd = prof["kernels"][dom]
    launches = max(kd["launches"], 1)
    avg_ms = kd["ms"] / launches
    bpl = kd["bytes"] / launches
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    per_kernel = [{"kernel": RATE_KERNELS[b], "launches": prof["kernels"][b]["launches"],
                   "ms_per_launch": prof["kernels"][b]["ms"] / max(prof["kernels"][b]["launches"], 1),
                   "GBps": (prof["kernels"][b]["bytes"] / (prof["kernels"][b]["ms"] * 1e-3) / 1e9)
                   if prof["kernels"][b]["ms"] > 0 else 0.0} for b in groups]
    traffic = traffic_for(RATE_KERNELS[dom], workload)
    rl = {"bound": "hbm", "kernel": RATE_KERNELS[dom], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
          "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
          "bytes_per_launch": bpl, "avg_launch_ms": avg_ms, "launches": launches,
          "rounds": prof["kernel_launches"]}
    if traffic and avg_ms > 0:
        # the bytes the memory interface actually moved (whole lines for the
        # 4-byte label gathers), over the same launch duration
        rl["traffic_GBps"] = traffic / (avg_ms * 1e-3) / 1e9
        rl["traffic_frac"] = rl["traffic_GBps"] / HBM_PEAK_GBS
    return rl, per_kernel


# Kernels of each launch group (the roofline groups above), and the kernels
# of an LP round as a whole, for the rocprofv3 counter summaries.
GROUP_KERNELS = [["k_rate_tiny", "k_rate_b32"], ["k_rate_small"], ["k_rate_mid"], ["k_rate_large"],
                 ["k_hub_prep", "k_hub_reuse", "k_hub_chunk", "k_hub_part", "k_hub_final"],
                 ["k_mark", "k_mark_big"]]
ROUND_KERNELS = {k for g in GROUP_KERNELS for k in g} | {
    "k_round_begin", "k_bin_count", "k_bin_write", "k_bin_scan1", "k_bin_totals", "k_conn_build", "k_conn_zero_hubs",
    "k_rate_cached", "k_incoming", "k_decide", "k_fold", "k_contended_small", "k_contended_split", "k_contended_mark",
    "k_contended_add", "k_ta_sums", "k_ta_scan_small", "k_ta_admit", "k_ta_reduce", "k_apply"}


def short_kernel_name(name: str) -> str:
    """sclap::k_rate_mid<true>(...) -> k_rate_mid; library kernels keep a
    short form of their name."""
    base = name.split("(")[0].replace("void ", "").strip()
    if "rocprim" in base:
        return "rocprim " + base.split("detail::")[-1].split("<")[0]
    return base.split("::")[-1].split("<")[0]


def summarize_counters(a) -> int:
    """Summary of rocprofv3 runs of the same bench command: the kernel trace
    (durations), a FETCH_SIZE and a WRITE_SIZE counter run, and the two
    counter runs of a plain device copy of --calib-copy-mb MiB (the scale of
    each counter).  Writes profiles/traffic.json (HBM bytes per launch of
    every roofline group, for the current kernel sources) and prints a
    markdown table."""
    import csv
    import glob

    def rows(d, what):
        fs = glob.glob(os.path.join(d, "**", f"*{what}.csv"), recursive=True)
        if not fs:
            raise SystemExit(f"no *{what}.csv under {d}")
        return list(csv.DictReader(open(fs[0])))

    def per_kernel(d, what):
        out = {}
        for r in rows(d, what):
            k = short_kernel_name(r["Kernel_Name"])
            out.setdefault(k, [0, 0.0])
            out[k][0] += 1
            out[k][1] += float(r["Counter_Value"])
        return out

    copy_bytes = a.calib_copy_mb * (1 << 20)
    cf = [float(r["Counter_Value"]) for r in rows(a.calib_fetch, "counter_collection")
          if "copyBuffer" in r["Kernel_Name"]]
    cw = [float(r["Counter_Value"]) for r in rows(a.calib_write, "counter_collection")
          if "copyBuffer" in r["Kernel_Name"]]
    f_factor = copy_bytes / (sum(cf) / len(cf) * 1024.0)
    w_factor = copy_bytes / (sum(cw) / len(cw) * 1024.0)
    fetch = per_kernel(a.fetch, "counter_collection")
    write = per_kernel(a.write, "counter_collection")
    dur = {}
    for r in rows(a.trace, "kernel_trace"):
        k = short_kernel_name(r["Kernel_Name"])
        dur.setdefault(k, [0, 0.0])
        dur[k][0] += 1
        dur[k][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    # the bench's JSON line among the lines the profiled run printed
    line = next(json.loads(x) for x in reversed(open(a.bench_line).read().splitlines()) if x.startswith("{"))
    launches = [rk["launches"] for rk in line["rating_kernels"]]

    def agg(names):
        fb = sum(fetch.get(k, [0, 0.0])[1] for k in names) * 1024.0 * f_factor
        wb = sum(write.get(k, [0, 0.0])[1] for k in names) * 1024.0 * w_factor
        ms = sum(dur.get(k, [0, 0.0])[1] for k in names)
        nd = sum(dur.get(k, [0, 0.0])[0] for k in names)
        return fb, wb, ms, nd

    groups = {}
    print("| kernels | dispatches | fetched GB | written GB | kernel ms | GB/s | of 8 TB/s |")
    print("|---|---:|---:|---:|---:|---:|---:|")

    def row(label, names):
        fb, wb, ms, nd = agg(names)
        rate = (fb + wb) / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        print(f"| {label} | {nd} | {fb / 1e9:.2f} | {wb / 1e9:.2f} | {ms:.2f} | {rate:.0f} | "
              f"{100.0 * rate / HBM_PEAK_GBS:.1f}% |")
        return fb, wb, ms, nd

    for i, names in enumerate(GROUP_KERNELS):
        fb, wb, ms, nd = row(RATE_KERNELS[i], names)
        la = max(launches[i] * a.partitions, 1)
        groups[RATE_KERNELS[i]] = {"dispatches": nd, "fetch_bytes_per_launch": fb / la,
                                   "write_bytes_per_launch": wb / la, "bytes_per_launch": (fb + wb) / la,
                                   "kernels": names}
    row("LP rounds (all round kernels)", sorted(ROUND_KERNELS))
    others = sorted(k for k in dur if k not in ROUND_KERNELS)
    row("everything else (contraction, initial partition, cut, copies)", others)
    row("rocPRIM (contraction sorts, reductions, scans)", [k for k in others if k.startswith("rocprim")])
    if a.write_traffic:
        out = {"workload": a.traffic_key, "source_digest": kernel_source_digest(),
               "digest_files": ["paper_1402_3281_amd/csrc/common.h", "paper_1402_3281_amd/csrc/lp_kernels.hip"],
               "calibration": {"copy_bytes": copy_bytes, "fetch_factor": f_factor, "write_factor": w_factor},
               "partitions": a.partitions, "kernels": groups}
        json.dump(out, open(os.path.join(ROOT, "profiles", "traffic.json"), "w"), indent=1)
    return 0


def profiled(ctx, fn):
    """Run fn once more with HIP events around every rating launch."""
    import torch

    ctx.profile(True)
    fn()
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    return prof


def visits_of(st: dict) -> int:
    return sum(st["visits_c"]) + sum(st["visits_r"])


def round_rate(prof: dict):
    return (prof["visits"] / (prof["round_ms"] * 1e-3)) if prof["round_ms"] > 0 else None


def base_line(metric, value, unit, steps, warmup, ms_per_step, config, scaling="weak"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": scaling, "vs_baseline": None,
            "dtype": "int32", "data": "synthetic", "config": config}


# --------------------------------------------------------------------------
# R-MAT s22 + RGG 2^22, k = 16 (default)

def run_two_graphs(args) -> int:
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
    sts = []
    for i in range(args.steps):
        sts = step()
        visits += sum(visits_of(s) for s in sts)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = profiled(ctx, step)
    rl, per_kernel = roofline(prof, "two-graphs-s22")

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
            r = oracle.cluster(og, U, 10, 0, 1)
            cv += r.visits
            rounds += r.rounds
        ct = time.perf_counter() - t1
        cpu = {"value": cv / ct, "unit": "edge visits/s", "cores": 1, "kind": "oracle",
               "sample": "oracle level-0 clustering of both graphs, exactly 10 LP rounds each (no stop rule), "
                         f"single thread, gcc -O2: {rounds} rounds, {cv} visits in {ct:.1f}s", **host_info()}

    line = base_line(
        "SCLaP edge visits/s (multilevel partition, clustering + refinement rounds)", visits / elapsed,
        "edge visits/s", args.steps, args.warmup, elapsed * 1000.0 / args.steps,
        {"workload": f"rmat-s{scale}-ef16 + rgg-2^{scale}-d10, k=16, eps=3/100, f=14, coarsen to <= {thr}, "
                     "10 LP rounds per level, LP refinement on every level",
         "k": k, "graphs": [{"name": g.name, "n": g.n, "m": g.m} for g in graphs],
         "cuts": [s["cut"] for s in sts], "levels": [s["n_level"] for s in sts]})
    line.update({
        "sclap_round_visits_per_s": round_rate(prof),
        "visits_per_step": visits // max(args.steps, 1),
        "phase_ms": [dict(graph=g.name, **s["ms"]) for g, s in zip(graphs, sts)],
        "rating_kernels": per_kernel,
        "roofline": rl,
        "cpu_baseline": cpu,
    })
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


# --------------------------------------------------------------------------
# The Section 4 extensions on R-MAT s22 + RGG 2^22

EXT_CONFIGS = [
    ("plain", {}),
    ("V2 (2 V-cycles)", {"vcycles": 2}),
    ("V3 (3 V-cycles)", {"vcycles": 3}),
    ("S4 (4 degree-ordered sub-rounds)", {"subrounds": 4}),
    ("E3 (3-member ensemble)", {"ensemble": 3}),
    ("B (extra coarse imbalance 1/10)", {"delta": (1, 10)}),
    ("V3/B/S4", {"vcycles": 3, "delta": (1, 10), "subrounds": 4}),
]


def run_extensions(args) -> int:
    """Every extension configuration partitions both graphs `steps` times
    after `warmup` untimed runs; reported per configuration: time per
    step, edge visits/s and the cuts against the plain scheme's.  value: the
    edge visits/s of three V-cycles (the paper's V configuration)."""
    import torch

    import graphgen
    import paper_1402_3281_amd as sc

    k, thr, scale = 16, 80000, args.scale
    t0 = time.time()
    graphs = [graphgen.rmat(scale, 16, seed=1), graphgen.rgg(1 << scale, 10.0, seed=1)]
    log(f"generated inputs in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    devs = [sc.DeviceGraph.from_host(g, rows_sorted=True) for g in graphs]
    parts = [torch.empty(g.n, dtype=torch.int32, device="cuda") for g in graphs]
    ctx = sc.Context(0)
    stream = torch.cuda.current_stream()
    rows = []
    plain_cuts = None
    for name, kw in EXT_CONFIGS:
        def step():
            return [sc.partition(ctx, d, k, threshold=thr, stream=stream, part_out=p, **kw)[1]
                    for d, p in zip(devs, parts)]

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        visits, sts = 0, []
        for _ in range(args.steps):
            sts = step()
            visits += sum(sum(s["cycles"]["visits"]) for s in sts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        cuts = [s["cut"] for s in sts]
        if plain_cuts is None:
            plain_cuts = cuts
        row = {"config": name, "params": {a: list(b) if isinstance(b, tuple) else b for a, b in kw.items()},
               "ms_per_step": el * 1000.0 / args.steps, "visits_per_s": visits / el, "cuts": cuts,
               "cut_vs_plain": [c / p for c, p in zip(cuts, plain_cuts)],
               "max_block_le_lmax": [s["max_block"] <= s["lmax"] for s in sts],
               "cycle_cuts": [s["cycles"]["cut"] for s in sts]}
        rows.append(row)
        log(f"{name}: {row['ms_per_step']:.1f} ms, cuts {cuts}")
    v3 = next(r for r in rows if r["config"].startswith("V3 "))
    line = base_line("SCLaP edge visits/s (multilevel partition with three V-cycles)", v3["visits_per_s"],
                     "edge visits/s", args.steps, args.warmup, v3["ms_per_step"],
                     {"workload": f"rmat-s{scale}-ef16 + rgg-2^{scale}-d10, k=16, eps=3/100, f=14, coarsen to <= "
                                  f"{thr}, 10 LP rounds per level, LP refinement on every level; Section 4 "
                                  "extensions", "k": k, "graphs": [{"name": g.name, "n": g.n, "m": g.m} for g in graphs]})
    line["configs"] = rows
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


# --------------------------------------------------------------------------
# 512 mixed graphs: batched versus plain

def run_batch(args) -> int:
    import numpy as np
    import torch

    import graphgen
    import paper_1402_3281_amd as sc

    t0 = time.time()
    specs = graphgen.batch_specs(count=args.graphs, seed=3)
    graphs = [s.make() for s in specs]
    ks = [s.k for s in specs]
    log(f"generated {len(graphs)} graphs in {time.time() - t0:.1f}s: n={sum(g.n for g in graphs)} "
        f"m={sum(g.m for g in graphs)}")
    torch.cuda.set_device(0)
    devs = [sc.DeviceGraph.from_host(g, rows_sorted=True) for g in graphs]
    ctx = sc.Context(0)
    stream = torch.cuda.current_stream()
    plain_parts = [torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in graphs]
    batch_parts = [torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in graphs]

    def plain():
        return [sc.partition(ctx, d, k, stream=stream, part_out=p)[1] for d, k, p in zip(devs, ks, plain_parts)]

    def batched():
        return sc.partition_batch(ctx, devs, ks, stream=stream, parts_out=batch_parts)[1]

    def timed(fn, name):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = None
        for _ in range(args.steps):
            out = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / args.steps
        log(f"{name}: {dt * 1e3:.1f} ms per pass over the batch")
        return dt, out

    tune = None
    if not args.no_autotune:
        # the degree bins' bounds, tuned on the batch's largest graph (untimed setup)
        big = max(range(len(graphs)), key=lambda i: graphs[i].m)
        _, _, U = sc.bounds(graphs[big].n, 1, ks[big], (3, 100), 14)
        tune = ctx.autotune(devs[big], U, rounds=3, stream=stream)
        log(f"autotuned bin bounds {tune}")
    tp, sts_p = timed(plain, "plain")
    tb, sts_b = timed(batched, "batched")
    same = all(torch.equal(a[:g.n], b[:g.n]) for a, b, g in zip(plain_parts, batch_parts, graphs))
    same = same and all(a["cut"] == b["cut"] for a, b in zip(sts_p, sts_b))
    visits = sum(visits_of(s) for s in sts_b)
    prof = profiled(ctx, batched)
    rl, per_kernel = roofline(prof, "batch-512")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t1 = time.perf_counter()
        done = 0
        equal = True
        while done < len(graphs) and time.perf_counter() - t1 < 15.0:
            part, st = oracle.partition(graphs[done], ks[done])
            equal = equal and st["cut"] == sts_b[done]["cut"] and np.array_equal(
                part, batch_parts[done][:graphs[done].n].cpu().numpy())
            done += 1
        ct = time.perf_counter() - t1
        cpu = {"value": done / ct, "unit": "graphs/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle partition of the first {done} graphs of the batch, one after the other, single "
                         f"thread; blocks equal to the batched GPU blocks: {equal}", **host_info()}

    line = base_line(
        "graphs/s, mixed graphs partitioned batched (every executor step fused over all graphs)",
        len(graphs) / tb, "graphs/s", args.steps, args.warmup, tb * 1000.0,
        {"workload": f"{len(graphs)} graphs, n log-uniform in [2^8, 2^16], half R-MAT (edge factor 4-32), half "
                     "RGG (degree 6-12), k in {2,4,8,16}, eps=3/100, f=14, coarsening threshold max(60k, n/(60k))",
         "graphs": len(graphs), "n_total": sum(g.n for g in graphs), "m_total": sum(g.m for g in graphs)})
    line.update({
        "plain": {"graphs_per_s": len(graphs) / tp, "ms_per_pass": tp * 1e3,
                  "visits_per_s": sum(visits_of(s) for s in sts_p) / tp},
        "batched": {"graphs_per_s": len(graphs) / tb, "ms_per_pass": tb * 1e3, "visits_per_s": visits / tb},
        "batched_over_plain": tp / tb,
        "identical_results": bool(same),
        "sclap_round_visits_per_s": round_rate(prof),
        "rating_kernels": per_kernel,
        "autotune": tune,
        "roofline": rl,
        "cpu_baseline": cpu,
    })
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0 if same else 1


# --------------------------------------------------------------------------
# served Poisson stream versus plain

def run_serve(args) -> int:
    import threading

    import numpy as np
    import torch

    import graphgen
    import paper_1402_3281_amd as sc

    specs = graphgen.serve_specs(count=args.jobs, seed=4)
    pool_n = min(args.pool, len(specs))
    t0 = time.time()
    pool = [specs[i].make() for i in range(pool_n)]
    log(f"generated a pool of {pool_n} graphs in {time.time() - t0:.1f}s: n={sum(g.n for g in pool)} "
        f"m={sum(g.m for g in pool)}")
    torch.cuda.set_device(0)
    devs = [sc.DeviceGraph.from_host(g, rows_sorted=True) for g in pool]
    # job i partitions pool graph (i mod pool size) into its own k
    jobs = [(i % pool_n, specs[i].k) for i in range(len(specs))]
    ctx = sc.Context(0)
    stream = torch.cuda.current_stream()
    outs = [torch.empty(max(pool[g].n, 1), dtype=torch.int32, device="cuda") for g, _ in jobs]

    # plain: one job after the other, on a prefix of the stream
    n_plain = min(args.plain_jobs, len(jobs))
    plain_parts = [torch.empty(max(pool[g].n, 1), dtype=torch.int32, device="cuda") for g, _ in jobs[:n_plain]]
    for g, k in jobs[:min(4, n_plain)]:
        sc.partition(ctx, devs[g], k, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_cut = []
    for (g, k), p in zip(jobs[:n_plain], plain_parts):
        plain_cut.append(sc.partition(ctx, devs[g], k, stream=stream, part_out=p)[1]["cut"])
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    plain_jps = n_plain / tp
    log(f"plain: {n_plain} jobs in {tp:.2f}s ({plain_jps:.1f} jobs/s)")

    budget = args.budget_gb << 30
    # the plain runs' cached device blocks would sit beside the server's
    # budget: hand them back to HIP first
    torch.cuda.synchronize()
    ctx.trim()

    def serve(rate: float, count: int):
        srv = sc.Server(ctx, hbm_budget_bytes=budget, max_active=args.max_active)
        arrivals = graphgen.poisson_arrivals(count, rate, seed=5) if rate > 0 else np.zeros(count)
        tickets = [None] * count
        ready = threading.Semaphore(0)
        t_start = time.perf_counter()

        def submitter():
            for i in range(count):
                dt = arrivals[i] - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
                g, k = jobs[i]
                tickets[i] = srv.submit(devs[g], k, outs[i])
                ready.release()

        th = threading.Thread(target=submitter)
        th.start()
        res = []
        for i in range(count):
            ready.acquire()
            res.append(srv.wait(tickets[i]))
            if (i + 1) % 1000 == 0:
                log(f"  {i + 1} jobs done")
        th.join()
        wall = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        return res, st, wall

    # capacity: every job of a prefix submitted at once
    n_cap = min(args.capacity_jobs, len(jobs))
    _, _, wall = serve(0.0, n_cap)
    capacity = n_cap / wall
    log(f"closed loop: {n_cap} jobs in {wall:.2f}s ({capacity:.1f} jobs/s)")
    rate = args.rate if args.rate > 0 else 0.8 * capacity
    res, st, wall = serve(rate, len(jobs))
    log(f"Poisson stream at {rate:.1f} jobs/s: {len(jobs)} jobs in {wall:.2f}s, p50 {st['p50_ms']:.1f} ms "
        f"p99 {st['p99_ms']:.1f} ms")
    ok = all(r["status"] == sc.OK for r in res)
    same = all(res[i]["cut"] == plain_cut[i] and torch.equal(outs[i][:pool[jobs[i][0]].n],
                                                              plain_parts[i][:pool[jobs[i][0]].n])
               for i in range(n_plain))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        t1 = time.perf_counter()
        done = 0
        while done < len(jobs) and time.perf_counter() - t1 < 15.0:
            g, k = jobs[done]
            oracle.partition(pool[g], k)
            done += 1
        ct = time.perf_counter() - t1
        cpu = {"value": done / ct, "unit": "jobs/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle partition of the first {done} jobs of the stream, one after the other, single thread",
               **host_info()}

    line = base_line(
        "jobs/s, served Poisson stream of partition jobs (continuous batching under an HBM budget)",
        st["jobs_per_s"], "jobs/s", 1, 0, wall * 1000.0,
        {"workload": f"{len(jobs)} jobs, n log-uniform in [2^10, 2^20], R-MAT (edge factor 16) and RGG (degree 8) "
                     f"1:1, k in 2..64, graphs from a pool of the first {pool_n} job graphs, Poisson arrivals at "
                     f"{rate:.1f} jobs/s, HBM budget {args.budget_gb} GB",
         "jobs": len(jobs), "pool": pool_n, "rate_per_s": rate, "budget_gb": args.budget_gb}, scaling="strong")
    line.update({
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "completed": st["completed"], "peak_bytes": st["peak_bytes"],
        "closed_loop_jobs_per_s": capacity, "plain_jobs_per_s": plain_jps, "plain_jobs": n_plain,
        "served_over_plain": st["jobs_per_s"] / plain_jps, "all_ok": ok, "identical_to_plain": bool(same),
        "cpu_baseline": cpu,
    })
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0 if (ok and same) else 1


# --------------------------------------------------------------------------
# R-MAT scale 26, k = 32

def run_large(args) -> int:
    import numpy as np
    import torch

    import graphgen
    import paper_1402_3281_amd as sc

    k, scale = 32, args.scale
    t0 = time.time()
    graphgen.set_progress(True)
    g = graphgen.rmat(scale, 16, seed=1)
    graphgen.set_progress(False)
    log(f"generated {g.name} n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    torch.cuda.set_device(0)
    dev = sc.DeviceGraph.from_host(g, rows_sorted=True)
    part = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ctx = sc.Context(0)
    stream = torch.cuda.current_stream()
    tune = None
    if not args.no_autotune:
        # the degree bins' bounds, picked by timing clustering rounds (untimed setup)
        _, _, U = sc.bounds(g.n, 1, k, (3, 100), 14)
        tune = ctx.autotune(dev, U, rounds=3, stream=stream)
        log(f"autotuned bin bounds {tune}")

    def step():
        return sc.partition(ctx, dev, k, stream=stream, part_out=part)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = None
    visits = 0
    for i in range(args.steps):
        st = step()
        visits += visits_of(st)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    prof = profiled(ctx, step)
    rl, per_kernel = roofline(prof, f"rmat-s{scale}")

    # properties that hold at any size: the cut and block weights recomputed on
    # the host from the returned blocks, every block within L_max
    log("checking result properties on the host")
    p = part.cpu().numpy()
    lmax, _, _ = sc.bounds(g.n, 1, k, (3, 100), 14)
    bw = np.bincount(p, minlength=k)
    cut = 0
    step_rows = 1 << 22
    for lo in range(0, g.n, step_rows):
        hi = min(g.n, lo + step_rows)
        a, b = int(g.row_ptr[lo]), int(g.row_ptr[hi])
        src = np.repeat(p[lo:hi], np.diff(g.row_ptr[lo:hi + 1]))
        cut += int(np.count_nonzero(src != p[g.col[a:b]]))
    cut //= 2
    props = {"blocks_in_range": bool(p.min() >= 0 and p.max() < k), "max_block": int(bw.max()), "lmax": lmax,
             "max_block_le_lmax": bool(bw.max() <= lmax), "max_block_matches": int(bw.max()) == st["max_block"],
             "cut_recomputed": cut, "cut_matches": cut == st["cut"]}
    ok = props["blocks_in_range"] and props["max_block_le_lmax"] and props["max_block_matches"] and \
        props["cut_matches"]
    log(f"properties: {props}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        log("timing the oracle")
        t1 = time.perf_counter()
        _, _, U = oracle.bounds(g.n, 1, k, 3, 100, 14)
        r = oracle.cluster(oracle.OGraph.of(g), U, 1, 0, 1)
        ct = time.perf_counter() - t1
        cpu = {"value": r.visits / ct, "unit": "edge visits/s", "cores": 1, "kind": "oracle",
               "sample": f"oracle clustering round 1 on level 0, single thread: {r.visits} visits in {ct:.1f}s",
               **host_info()}

    line = base_line(
        "SCLaP edge visits/s (multilevel partition, clustering + refinement rounds)", visits / elapsed,
        "edge visits/s", args.steps, args.warmup, elapsed * 1000.0 / args.steps,
        {"workload": f"rmat-s{scale}-ef16, k={k}, eps=3/100, f=14, coarsening threshold max(60k, n/(60k)), "
                     "10 LP rounds per level, LP refinement on every level",
         "k": k, "graphs": [{"name": g.name, "n": g.n, "m": g.m}], "cut": st["cut"], "levels": st["n_level"]})
    line.update({
        "sclap_round_visits_per_s": round_rate(prof),
        "phase_ms": st["ms"],
        "properties": props,
        "autotune": tune,
        "rating_kernels": per_kernel,
        "roofline": rl,
        "cpu_baseline": cpu,
    })
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0 if ok else 1


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=("large", "two-graphs", "batch", "serve", "extensions"),
                    help="large: R-MAT s26, k=32 (default); two-graphs: R-MAT s22 + RGG 2^22, k=16; batch: 512 "
                         "mixed graphs batched vs plain; serve: Poisson stream of jobs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default degree-bin bounds (large, batch)")
    ap.add_argument("--scale", type=int, default=0, help="R-MAT scale (two-graphs: 22, large: 26)")
    ap.add_argument("--graphs", type=int, default=512, help="batch size (batch)")
    ap.add_argument("--jobs", type=int, default=10000, help="jobs in the served stream (serve)")
    ap.add_argument("--pool", type=int, default=1024, help="distinct graphs the served jobs draw from (serve)")
    ap.add_argument("--plain-jobs", type=int, default=1000, help="jobs run one by one for comparison (serve)")
    ap.add_argument("--capacity-jobs", type=int, default=2000, help="jobs of the closed-loop capacity run (serve)")
    ap.add_argument("--rate", type=float, default=0.0, help="arrival rate in jobs/s (serve; default 0.8 x capacity)")
    ap.add_argument("--budget-gb", type=int, default=200, help="HBM budget of the server (serve)")
    ap.add_argument("--max-active", type=int, default=256, help="jobs on the device at once (serve)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--summarize", action="store_true",
                    help="summarise rocprofv3 runs (--trace, --fetch, --write, --calib-fetch, --calib-write, "
                         "--bench-line) instead of running")
    for opt in ("--trace", "--fetch", "--write", "--calib-fetch", "--calib-write", "--bench-line"):
        ap.add_argument(opt, default="")
    ap.add_argument("--partitions", type=int, default=2, help="partition steps in each profiled run (summarize)")
    ap.add_argument("--write-traffic", action="store_true", help="write profiles/traffic.json (summarize)")
    ap.add_argument("--traffic-key", default="rmat-s26",
                    help="workload key the bytes in profiles/traffic.json belong to (summarize)")
    args = ap.parse_args()
    if args.summarize:
        args.calib_copy_mb = args.calib_copy_mb or 1024
        return summarize_counters(args)
    if args.calib_copy_mb:
        return copy_calibration(args.calib_copy_mb)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the partitioner's multi-GPU path is "
              "not built.", file=sys.stderr)
        return 2
    if args.workload == "two-graphs":
        args.scale = args.scale or 22
        return run_two_graphs(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "extensions":
        args.scale = args.scale or 22
        return run_extensions(args)
    if args.workload == "serve":
        return run_serve(args)
    args.scale = args.scale or 26
    return run_large(args)


if __name__ == "__main__":
    sys.exit(main())
