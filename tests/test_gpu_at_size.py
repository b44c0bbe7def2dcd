"""Parity at the real sizes of the benchmark workloads, against digests the
oracle wrote (tests/golden/make_size_goldens.py, oracle only):

- the scale-22 R-MAT and 2^22 RGG graphs level by level: each level's
  clustering labels and the coarse CSR its contraction builds;
- the 512 mixed graphs of the batch workload, partitioned in one fused batch;
- 256 jobs of the served workload (up to 2^20 nodes), all on the device at
  once;
- the first three clustering rounds of the R-MAT scale-26 graph.

The path counters show that the fused rounds took the multi-job, device-wide
binning-scan and device-wide contended-admission paths."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    return json.load(open(os.path.join(GOLDEN, name)))


def digest(a, dtype="<i4") -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3281_amd as sc

    sc.load_library()
    return sc


@pytest.fixture(scope="module")
def ctx(sc):
    c = sc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("which", [0, 1])
def test_scale22_levels(sc, ctx, which):
    rec = gold("levels_s22.json")["graphs"][which]
    g = graphgen.config2_graphs()[which]
    assert g.name == rec["graph"]
    d = sc.DeviceGraph.from_host(g, rows_sorted=True)
    for i, lv in enumerate(rec["levels"]):
        print(f"{g.name} level {i}: n={lv['n']} m={lv['m']}", flush=True)
        assert (d.n, d.m) == (lv["n"], lv["m"])
        lab, nc, rs = sc.cluster(ctx, d, rec["U"], 10, 1, 1)
        assert digest(lab.cpu().numpy()) == lv["labels_sha256"], i
        assert rs["rounds"] == lv["rounds"] and rs["moved"] == lv["moved"] and rs["visits"] == lv["visits"], i
        cof, cg = sc.contract(ctx, d, lab, drop_isolated=(i == 0))
        h = cg.to_host()
        assert (cg.n, cg.m) == (lv["coarse_n"], lv["coarse_m"]), i
        assert digest(cof.cpu().numpy()) == lv["coarse_of_sha256"], i
        assert digest(h["row_ptr"], "<i8") == lv["row_ptr_sha256"], i
        assert digest(h["col"]) == lv["col_sha256"] and digest(h["ew"]) == lv["ew_sha256"], i
        assert digest(h["nw"], "<i8") == lv["nw_sha256"], i
        d = cg.to_device()
        cg.close()


def test_batch512(sc, ctx):
    rec = gold("batch512.json")
    specs = graphgen.batch_specs(512)
    graphs = [s.make() for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    before = ctx.path_counters()
    print("batch of 512 graphs", flush=True)
    parts, sts = sc.partition_batch(ctx, devs, [s.k for s in specs])
    after = ctx.path_counters()
    for g, p, st, want in zip(graphs, parts, sts, rec["graphs"]):
        assert g.name == want["graph"]
        assert digest(p.cpu().numpy()) == want["part_sha256"], g.name
        assert st["cut"] == want["cut"] and st["max_block"] == want["max_block"], g.name
        assert st["n_level"] == want["n_level"], g.name
        assert sum(st["visits_c"]) + sum(st["visits_r"]) == want["visits"], g.name
    delta = {k: after[k] - before[k] for k in after}
    print(delta, flush=True)
    assert delta["multi_job_rounds"] > 0 and delta["device_wide_bin_scans"] > 0


def test_served256_all_active(sc, ctx):
    rec = gold("served256.json")
    specs = graphgen.serve_specs(count=256, seed=61)
    graphs = [s.make() for s in specs]
    print(f"served: 256 jobs, {sum(g.n for g in graphs)} nodes", flush=True)
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    parts = [torch.full((g.n,), -1, dtype=torch.int32, device="cuda") for g in graphs]
    srv = sc.Server(ctx, hbm_budget_bytes=200 << 30, max_active=256)
    try:
        srv.hold(True)  # all 256 jobs are admitted together
        tickets = [srv.submit(d, s.k, p) for d, s, p in zip(devs, specs, parts)]
        srv.hold(False)
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
        paths = srv.path_counters()
    finally:
        srv.close()
    print(st, paths, flush=True)
    for g, p, r, want in zip(graphs, parts, results, rec["jobs"]):
        assert g.name == want["graph"]
        assert r["status"] == sc.OK, g.name
        assert digest(p.cpu().numpy()) == want["part_sha256"], g.name
        assert r["cut"] == want["cut"] and r["max_block"] == want["max_block"], g.name
    assert st["peak_active"] == 256
    assert paths["multi_job_rounds"] > 0 and paths["device_wide_bin_scans"] > 0
    assert paths["device_wide_contended"] > 0 and paths["hub_rounds"] > 0


def test_scale26_first_rounds(sc, ctx):
    rec = gold("s26_rounds.json")
    g = graphgen.rmat(26, 16, seed=1)
    assert g.name == rec["graph"] and g.col.shape[0] == rec["m"]
    d = sc.DeviceGraph.from_host(g, rows_sorted=True)
    del g
    print("R-MAT scale 26, three clustering rounds", flush=True)
    lab, nc, rs = sc.cluster(ctx, d, rec["U"], rec["rounds"], rec["stop_rule"], 1)
    assert rs["moved"] == rec["moved"] and rs["visits"] == rec["visits"]
    assert nc == rec["clusters"]
    assert digest(lab.cpu().numpy()) == rec["labels_sha256"]
