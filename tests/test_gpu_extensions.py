"""The Section 4 extensions on the GPU through the C ABI, element by element
against the oracle: partition-respecting clustering and iterated V-cycles
(Appendix B.1), extra coarse-level imbalance, degree-ordered sub-rounds and
ensemble clusterings with their overlay."""
import numpy as np
import pytest

import graphgen
import oracle
from tinygraphs import from_edges

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def weighted(g, seed):
    """The graph with random int32 edge weights (symmetric) and node weights."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lo = np.minimum(src, g.col).astype(np.int64)
    hi = np.maximum(src, g.col).astype(np.int64)
    ew = (((lo * 1000003 + hi) * 2654435761) % 7 + 1).astype(np.int32)
    nw = rng.integers(1, 5, g.n).astype(np.int64)
    return graphgen.Graph(g.row_ptr, g.col, ew=ew, nw=nw)


GRAPHS = [
    ("rmat12", lambda: graphgen.rmat(12, 8, seed=3)),
    ("rgg5000", lambda: graphgen.rgg(5000, 8.0, seed=4)),
    ("rmat11w", lambda: weighted(graphgen.rmat(11, 16, seed=6), 1)),
]


@pytest.mark.parametrize("name,make", GRAPHS)
@pytest.mark.parametrize("blocks,member,sub", [(True, 0, 0), (False, 3, 0), (False, 0, 3), (True, 2, 2)])
def test_cluster_ext_equals_oracle(sc, ctx, name, make, blocks, member, sub):
    g = make()
    d = sc.DeviceGraph.from_host(g)
    rng = np.random.default_rng(len(name) + member + sub)
    blk = rng.integers(0, 5, g.n).astype(np.int32) if blocks else None
    U = 40
    print(f"cluster_ext {name} blocks={blocks} member={member} sub={sub}", flush=True)
    lab, nc, rs = sc.cluster(ctx, d, U, max_rounds=10, stop_rule=1, subrounds=sub, member=member,
                             blocks=None if blk is None else torch.from_numpy(blk).cuda())
    want = oracle.cluster_ext(g, U, 10, 1, 1, vblk=blk, subrounds=sub,
                              lab0=None if member == 0 else oracle.member_labels(g.n, member))
    assert np.array_equal(lab.cpu().numpy(), want.labels)
    assert rs["rounds"] == want.rounds and rs["moved"] == want.moved and rs["visits"] == want.visits
    assert nc == len(np.unique(want.labels))


@pytest.mark.parametrize("n", [0, 1, 777, 100000])
def test_overlay_equals_oracle(sc, ctx, n):
    rng = np.random.default_rng(n)
    O = rng.integers(0, max(n, 1), n).astype(np.int32)
    C = rng.integers(0, max(n // 5, 1), n).astype(np.int32)
    print(f"overlay n={n}", flush=True)
    dO = torch.from_numpy(O.copy()).cuda()
    cnt = sc.overlay(ctx, dO, torch.from_numpy(C).cuda())
    want, wc = oracle.overlay(O, C)
    assert np.array_equal(dO.cpu().numpy(), want) and cnt == wc


EXT_CASES = [
    dict(vcycles=2), dict(vcycles=3), dict(subrounds=3), dict(ensemble=3), dict(delta=(1, 5)),
    dict(vcycles=2, subrounds=2, ensemble=2, delta=(1, 10)),
]


def oracle_kw(kw):
    return {"vcycles": kw.get("vcycles", 1), "subrounds": kw.get("subrounds", 0),
            "ensemble": kw.get("ensemble", 1), "delta": kw.get("delta", (0, 1))}


def assert_same(st, part, want, wst, wcy):
    assert np.array_equal(part, want)
    for f in ("cut", "max_block", "levels", "n_level", "m_level", "rounds_c", "moved_c", "visits_c", "rounds_r",
              "moved_r", "visits_r", "ip_cut", "lmax", "U"):
        assert st[f] == wst[f], f
    assert st["cycles"]["cut"] == wcy["cut"] and st["cycles"]["max_block"] == wcy["max_block"]
    assert st["cycles"]["visits"] == wcy["visits"] and st["cycles"]["best"] == wcy["best"]
    assert st["cycles"]["levels"] == wcy["levels"]


@pytest.mark.parametrize("name,k,make", [
    ("rmat13", 8, lambda: graphgen.rmat(13, 8, seed=1)),
    ("rgg2e14", 4, lambda: graphgen.rgg(1 << 14, 8.0, seed=2)),
    ("rmat12ef16", 16, lambda: graphgen.rmat(12, 16, seed=5)),
    ("rmat11w", 4, lambda: weighted(graphgen.rmat(11, 8, seed=9), 2)),
])
@pytest.mark.parametrize("kw", EXT_CASES, ids=lambda kw: "-".join(f"{a}{b}" for a, b in kw.items()))
def test_partition_ext_equals_oracle(sc, ctx, name, k, make, kw):
    g = make()
    d = sc.DeviceGraph.from_host(g)
    print(f"partition_ext {name} k={k} {kw}", flush=True)
    part, st = sc.partition(ctx, d, k, **kw)
    want, wst, wcy = oracle.partition_ext(g, k, **oracle_kw(kw))
    assert_same(st, part.cpu().numpy(), want, wst, wcy)


def test_vcycles_without_coarsening(sc, ctx):
    """A threshold above n: every cycle refines level 0 only, later cycles
    from the best partition so far (isolated nodes set aside again)."""
    g = graphgen.rmat(10, 4, seed=4)
    d = sc.DeviceGraph.from_host(g)
    part, st = sc.partition(ctx, d, 4, threshold=1 << 20, vcycles=3)
    want, wst, wcy = oracle.partition_ext(g, 4, threshold=1 << 20, vcycles=3)
    assert_same(st, part.cpu().numpy(), want, wst, wcy)


def test_vcycle_hand_worked_on_gpu(sc, ctx):
    import json
    import os

    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "vcycle_example.json")))
    g = from_edges(d["graph"]["n"], d["graph"]["edges"])
    dg = sc.DeviceGraph.from_host(g)
    part, st = sc.partition(ctx, dg, d["k"], eps=tuple(d["eps"]), f=d["f"], threshold=d["threshold"], vcycles=2)
    assert part.cpu().numpy().tolist() == d["cycle2"]["part"]
    assert st["cycles"]["cut"] == [d["cycle1"]["cut"], d["cycle2"]["cut"]]
    assert st["cycles"]["visits"] == d["cycle_visits"] and st["cycles"]["best"] == d["best"]
    assert st["moved_c"][0] == d["cycle2"]["moved_c"] and st["visits_r"] == d["cycle2"]["visits_r"]


def test_empty_graph_with_extensions(sc, ctx):
    g = graphgen.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
    d = sc.DeviceGraph.from_host(g)
    part, st = sc.partition(ctx, d, 4, vcycles=3, subrounds=2, ensemble=2, delta=(1, 4))
    assert st["cut"] == 0 and st["cycles"]["cycles"] == 1


def test_batch_with_vcycles_equals_oracle(sc, ctx):
    specs = graphgen.batch_specs(count=8, seed=33, lg_lo=8, lg_hi=12)
    graphs = [s.make() for s in specs]
    ks = [s.k for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    parts, sts = sc.partition_batch(ctx, devs, ks, vcycles=2, subrounds=2)
    for g, k, p, st in zip(graphs, ks, parts, sts):
        want, wst, wcy = oracle.partition_ext(g, k, vcycles=2, subrounds=2)
        assert_same(st, p.cpu().numpy(), want, wst, wcy)


def test_served_jobs_with_extensions(sc, ctx):
    specs = graphgen.serve_specs(count=6, seed=51, lg_lo=9, lg_hi=13)
    graphs = [s.make() for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    parts = [torch.full((g.n,), -1, dtype=torch.int32, device="cuda") for g in graphs]
    kws = [dict(vcycles=2), dict(ensemble=2), dict(subrounds=3), dict(delta=(1, 5)), dict(vcycles=2, ensemble=2),
           {}]
    srv = sc.Server(ctx, hbm_budget_bytes=8 << 30, max_active=6)
    try:
        tickets = [srv.submit(d, s.k, p, **kw) for d, s, p, kw in zip(devs, specs, parts, kws)]
        results = [srv.wait(t) for t in tickets]
        for g, s, p, r, kw in zip(graphs, specs, parts, results, kws):
            assert r["status"] == sc.OK, g.name
            want, wst, _ = oracle.partition_ext(g, s.k, **oracle_kw(kw))
            assert np.array_equal(p.cpu().numpy(), want), (g.name, kw)
            assert r["cut"] == wst["cut"]
    finally:
        srv.close()
