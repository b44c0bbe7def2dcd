"""Write tests/golden/full_size.json: the oracle's results on the full-size
workloads (R-MAT scale 22 edge factor 16 and RGG 2^22 degree 10, k = 16,
coarsening to <= 80,000 nodes; R-MAT scale 14 clustering with U = 602).

Calls only the input generators and the oracle.  Partitions are stored as
SHA-256 digests of their int32 little-endian bytes next to the oracle's
statistics.  Takes a few minutes (single-threaded oracle).
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def main():
    out = {"source": "tests/golden/make_full_size.py (oracle only)", "partition": [], "cluster": []}
    g = graphgen.config1_graph()
    r = oracle.cluster(g, 602, 10, 0, 1)
    co = oracle.contract(g, r.labels)
    out["cluster"].append({"graph": g.name, "U": 602, "rounds": 10, "labels_sha256": digest(r.labels),
                           "moved": r.moved, "visits": r.visits, "coarse_n": int(co.n), "coarse_m": int(co.col.shape[0]),
                           "coarse_of_sha256": digest(co.coarse_of), "coarse_col_sha256": digest(co.col),
                           "coarse_ew_sha256": digest(co.ew), "cluster_cut": int(co.ew.sum()) // 2})
    for g in graphgen.config2_graphs():
        t = time.time()
        part, st = oracle.partition(g, 16, threshold=80000)
        st["part_sha256"] = digest(part)
        st["graph"] = g.name
        st["k"] = 16
        st["threshold_arg"] = 80000
        st["oracle_seconds_here"] = round(time.time() - t, 1)
        out["partition"].append(st)
        print(g.name, st["cut"], st["oracle_seconds_here"], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
