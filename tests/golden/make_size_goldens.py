"""Write the oracle's results at the benchmark workloads' real sizes, as
SHA-256 digests of int32/int64 little-endian arrays plus statistics:

  levels   tests/golden/levels_s22.json: the R-MAT scale-22 (edge factor 16)
           and RGG 2^22 (degree 10) graphs, k = 16: clustering with the 5%
           rule and U of the partition, contraction dropping the degree-0
           nodes on the input, repeated on every coarse level down to the
           partition's coarsening threshold (80,000 nodes): each level's
           labels, coarse_of and coarse CSR (row_ptr, col, edge and node
           weights);
  batch    tests/golden/batch512.json: the 512 mixed graphs of the batch
           workload (n log-uniform in [2^8, 2^16]), each partitioned alone;
  served   tests/golden/served256.json: 256 jobs of the served workload
           (n log-uniform in [2^10, 2^20], R-MAT edge factor 16 and RGG
           degree 8 alternating, k in 2..64), each partitioned alone;
  s26      tests/golden/s26_rounds.json: the first three clustering rounds
           (no stop rule) of the R-MAT scale-26 graph (k = 32, U = 154,290).

Calls only the input generators and the oracle (single-threaded; the batch
and served sets run several oracle processes side by side).  Usage:
python tests/golden/make_size_goldens.py levels batch served s26
"""
import hashlib
import json
import os
import sys
import time
import multiprocessing as mp

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def digest(a, dtype="<i4") -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def write(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


def levels():
    out = {"source": "tests/golden/make_size_goldens.py levels (oracle only)", "graphs": []}
    for g in graphgen.config2_graphs():
        t = time.time()
        lmax, W, U = oracle.bounds(int(g.node_weights().sum()), int(g.node_weights().max()), 16, 3, 100, 14)
        rec = {"graph": g.name, "k": 16, "U": U, "threshold": 80000, "levels": []}
        cur = g
        drop = 1
        while True:
            r = oracle.cluster(cur, U, 10, 1, 1)
            c = oracle.contract(cur, r.labels, drop)
            rec["levels"].append({
                "n": int(cur.n), "m": int(cur.col.shape[0]), "rounds": r.rounds, "moved": r.moved,
                "visits": r.visits, "labels_sha256": digest(r.labels), "coarse_of_sha256": digest(c.coarse_of),
                "coarse_n": int(c.n), "coarse_m": int(c.col.shape[0]),
                "row_ptr_sha256": digest(c.row_ptr, "<i8"), "col_sha256": digest(c.col),
                "ew_sha256": digest(c.ew), "nw_sha256": digest(c.nw, "<i8")})
            n_prev = int(cur.n) if not drop else int(np.count_nonzero(np.diff(cur.row_ptr)))
            cur = graphgen.Graph(c.row_ptr, c.col, ew=c.ew, nw=c.nw)
            drop = 0
            if cur.n <= 80000 or 20 * (n_prev - cur.n) < n_prev:
                break
        rec["oracle_seconds_here"] = round(time.time() - t, 1)
        out["graphs"].append(rec)
        print(g.name, [lv["coarse_n"] for lv in rec["levels"]], rec["oracle_seconds_here"], flush=True)
    write("levels_s22.json", out)


def _one(spec):
    g = spec.make()
    part, st = oracle.partition(g, spec.k)
    return {"graph": g.name, "n": int(g.n), "m": int(g.col.shape[0]), "k": spec.k, "part_sha256": digest(part),
            "cut": st["cut"], "max_block": st["max_block"], "levels": st["levels"], "n_level": st["n_level"],
            "visits": int(sum(st["visits_c"]) + sum(st["visits_r"]))}


def batch():
    specs = graphgen.batch_specs(512)
    t = time.time()
    with mp.get_context("spawn").Pool(6) as p:
        res = p.map(_one, specs, chunksize=4)
    write("batch512.json", {"source": "tests/golden/make_size_goldens.py batch (oracle only)",
                            "specs": "graphgen.batch_specs(512)", "graphs": res})
    print("batch", len(res), round(time.time() - t, 1), flush=True)


def served():
    specs = graphgen.serve_specs(count=256, seed=61)
    t = time.time()
    with mp.get_context("spawn").Pool(6) as p:
        res = p.map(_one, specs, chunksize=1)
    write("served256.json", {"source": "tests/golden/make_size_goldens.py served (oracle only)",
                             "specs": "graphgen.serve_specs(count=256, seed=61)", "jobs": res})
    print("served", len(res), round(time.time() - t, 1), flush=True)


def s26():
    t = time.time()
    g = graphgen.rmat(26, 16, seed=1)
    lmax, W, U = oracle.bounds(g.n, 1, 32, 3, 100, 14)
    r = oracle.cluster(g, U, 3, 0, 1)
    write("s26_rounds.json", {"source": "tests/golden/make_size_goldens.py s26 (oracle only)",
                              "graph": g.name, "n": int(g.n), "m": int(g.col.shape[0]), "U": U, "rounds": 3,
                              "stop_rule": 0, "labels_sha256": digest(r.labels), "moved": r.moved,
                              "visits": r.visits, "clusters": int(len(np.unique(r.labels))),
                              "oracle_seconds_here": round(time.time() - t, 1)})
    print("s26", r.moved, round(time.time() - t, 1), flush=True)


if __name__ == "__main__":
    for what in sys.argv[1:] or ["levels", "batch", "served", "s26"]:
        {"levels": levels, "batch": batch, "served": served, "s26": s26}[what]()
