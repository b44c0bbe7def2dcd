"""Parity of the gfx950 library with the CPU oracle, element by element.

Every call goes through the C ABI (via the ctypes binding).  Integer results
must be bit-identical: labels, coarse ids, coarse CSR arrays, blocks, cuts,
per-round moved counts and edge visits.
"""
import random

import numpy as np
import pytest

import graphgen
import oracle
from tinygraphs import family, from_edges, star

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


def dev(sc, g):
    return sc.DeviceGraph.from_host(g)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def tiny_graphs():
    return [(name, g) for name, g in family(seed=5, count=50) if g.n > 0]


def mid_graphs():
    out = []
    for seed in (1, 2):
        out.append(("rmat12", graphgen.rmat(12, 8, seed=seed)))
    out.append(("rmat14", graphgen.rmat(14, 16, seed=3)))
    out.append(("rgg14", graphgen.rgg(1 << 14, 10.0, seed=4)))
    out.append(("rmat_n5000", graphgen.rmat(13, 6, seed=5, n=5000)))
    # a hub above the workgroup-table bin (degree > 4096)
    rng = random.Random(6)
    n = 12000
    edges = star(n)[:9000] + [(i, i + 1) for i in range(9000, n - 1)]
    edges += [(rng.randrange(1, n), rng.randrange(1, n)) for _ in range(20000)]
    edges = sorted({(min(a, b), max(a, b)) for a, b in edges if a != b})
    out.append(("hub9000", from_edges(n, edges)))
    return out


def weighted(g, seed):
    rng = np.random.default_rng(seed)
    # symmetric edge weights: weight of {u, v} from a hash of the pair
    u = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    a, b = np.minimum(u, v), np.maximum(u, v)
    ew = (1 + ((a * 1000003 + b * 7919 + seed) % 5)).astype(np.int32)
    nw = rng.integers(0, 5, size=g.n).astype(np.int64)
    return graphgen.Graph(g.row_ptr, g.col, ew=ew, nw=nw, name=g.name + "-w")


def assert_cluster_parity(sc, ctx, g, U, rounds, stop_rule=0, dr=1):
    want = oracle.cluster(g, U, rounds, stop_rule, dr)
    lab, ncl, rs = sc.cluster(ctx, dev(sc, g), U, rounds, stop_rule, dr)
    got = host(lab)
    assert np.array_equal(got, want.labels)
    assert rs["rounds"] == want.rounds
    assert rs["moved"] == want.moved
    assert rs["visits"] == want.visits
    assert ncl == len(set(want.labels.tolist()))
    return want.labels


def assert_contract_parity(sc, ctx, g, labels, drop):
    want = oracle.contract(g, labels, drop_isolated=drop)
    d = dev(sc, g)
    cof, cg = sc.contract(ctx, d, torch.from_numpy(labels).cuda(), drop_isolated=bool(drop))
    got = cg.to_host()
    assert np.array_equal(host(cof), want.coarse_of)
    assert np.array_equal(got["row_ptr"], want.row_ptr)
    assert np.array_equal(got["col"], want.col)
    assert np.array_equal(got["ew"], want.ew)
    assert np.array_equal(got["nw"], want.nw)
    cg.close()


def test_cluster_and_contract_tiny(sc, ctx):
    rng = random.Random(1)
    for name, g in tiny_graphs():
        c = g.node_weights()
        for U in (1, 2, 3, int(c.sum()) + 1, max(1, int(c.sum()) // 3)):
            for dr in (1, 0):
                labels = assert_cluster_parity(sc, ctx, g, U, 6, 0, dr)
            assert_contract_parity(sc, ctx, g, labels, drop=rng.randint(0, 1))


def test_stop_rule_tiny(sc, ctx):
    for name, g in tiny_graphs()[:30]:
        assert_cluster_parity(sc, ctx, g, 4, 10, stop_rule=1)


def test_initial_partition_tiny(sc, ctx):
    for name, g in tiny_graphs():
        for k in (1, 2, 3, 5):
            for skip in (0, 1):
                want = oracle.initial_partition(g, k, skip)
                got = host(sc.initial_partition(ctx, dev(sc, g), k, skip_isolated=bool(skip)))
                assert np.array_equal(got, want), (name, k, skip)


def test_refine_tiny(sc, ctx):
    rng = random.Random(3)
    for name, g in tiny_graphs():
        for k in (2, 3):
            part = np.array([rng.randrange(k) for _ in range(g.n)], np.int32)
            c = g.node_weights()
            for lmax in (max(1, int(c.sum()) // k), int(c.sum())):
                want, rounds, moved, visits = oracle.refine(g, part, k, lmax, 8)
                p = torch.from_numpy(part.copy()).cuda()
                _, rs = sc.refine(ctx, dev(sc, g), p, k, lmax, 8)
                assert np.array_equal(host(p), want), name
                assert rs["rounds"] == rounds and rs["moved"] == moved and rs["visits"] == visits, name


def test_cut_tiny(sc, ctx):
    rng = random.Random(4)
    for name, g in tiny_graphs():
        k = rng.randint(1, 4)
        part = np.array([rng.randrange(k) for _ in range(g.n)], np.int32)
        want, bw = oracle.cut(g, part, k)
        got, gbw = sc.cut(ctx, dev(sc, g), torch.from_numpy(part).cuda(), k)
        assert got == want and list(bw) == gbw


def assert_partition_parity(sc, ctx, g, k, **kw):
    want_part, want = oracle.partition(g, k, **kw)
    part, got = sc.partition(ctx, dev(sc, g), k, **kw)
    assert np.array_equal(host(part), want_part), g.name
    for f in ("levels", "n_level", "m_level", "rounds_c", "rounds_r", "moved_c", "moved_r", "visits_c", "visits_r",
              "lmax", "W", "U", "threshold", "n_isolated", "ip_cut", "cut", "max_block"):
        assert got[f] == want[f], (g.name, f, got[f], want[f])
    return got


def test_partition_tiny(sc, ctx):
    for name, g in tiny_graphs():
        for k in (1, 2, 3):
            assert_partition_parity(sc, ctx, g, k)


@pytest.mark.parametrize("idx", range(6))
def test_partition_mid(sc, ctx, idx):
    name, g = mid_graphs()[idx]
    for k in (2, 16):
        assert_partition_parity(sc, ctx, g, k)
    gw = weighted(g, idx)
    assert_partition_parity(sc, ctx, gw, 4)


@pytest.mark.parametrize("idx", [2, 5])
def test_partition_many_blocks(sc, ctx, idx):
    """k above the limit for kept block connections (64): refinement rates
    from the bins in every round and admits through the general path."""
    name, g = mid_graphs()[idx]
    assert_partition_parity(sc, ctx, g, 96)


def test_batch_mixed_block_counts(sc, ctx):
    """One fused batch whose refinement slots take both admission paths (k up
    to 64: block connections and tiles; k above: the general path)."""
    specs = graphgen.batch_specs(count=6, seed=5, lg_lo=10, lg_hi=13)
    graphs = [s.make() for s in specs]
    ks = [8, 96, 16, 80, 2, 70]
    devs = [dev(sc, g) for g in graphs]
    parts, sts = sc.partition_batch(ctx, devs, ks)
    for g, k, p, st in zip(graphs, ks, parts, sts):
        want_part, want = oracle.partition(g, k)
        assert np.array_equal(host(p), want_part), (g.name, k)
        assert st["cut"] == want["cut"] and st["moved_r"] == want["moved_r"], (g.name, k)


def test_config1_cluster_contract(sc, ctx):
    """R-MAT scale 14, edge factor 8, U = 602, exactly 10 rounds, then one
    contraction; the cluster cut is the coarse edge weight / 2."""
    g = graphgen.config1_graph()
    lmax, W, U = sc.bounds(g.n, 1, 2)
    assert (lmax, W, U) == (8437, 602, 602)
    labels = assert_cluster_parity(sc, ctx, g, U, 10, 0, 1)
    assert_contract_parity(sc, ctx, g, labels, drop=0)


def test_row_order_and_repeat_invariance(sc, ctx):
    g = graphgen.rmat(13, 8, seed=9)
    rng = np.random.default_rng(0)
    col = g.col.copy()
    for v in range(g.n):
        seg = col[g.row_ptr[v]:g.row_ptr[v + 1]]
        rng.shuffle(seg)
    g2 = graphgen.Graph(g.row_ptr, col)
    p1, s1 = sc.partition(ctx, dev(sc, g), 8)
    p2, s2 = sc.partition(ctx, dev(sc, g2), 8)
    p3, s3 = sc.partition(ctx, dev(sc, g), 8)
    a, b, c = host(p1), host(p2), host(p3)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    for f in ("moved_c", "moved_r", "cut"):
        assert s1[f] == s2[f] == s3[f]


def _hash32(x: int) -> int:
    """The library's integer mixer, used here only to pick adversarial ids."""
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def test_hub_labels_crowding_one_part(sc, ctx):
    """A hub whose 5000 neighbour labels all fall into one of its label parts
    (more than one part table holds): the part is taken in several passes and
    the result still equals the oracle."""
    leaves = []
    x = 0
    while len(leaves) < 5000:
        if (_hash32(x) >> 19) & 3 == 0:
            leaves.append(x)
        x += 1
    hub = x
    n = hub + 1
    edges = [(hub, v) for v in leaves]
    rng = random.Random(9)
    edges += [(leaves[i], leaves[i + 1]) for i in range(0, 4000, 7)]
    rest = [v for v in range(n - 1) if (_hash32(v) >> 19) & 3 != 0]
    edges += [(rest[i], rest[i + 1]) for i in range(0, len(rest) - 1, 2)]
    g = from_edges(n, edges, rng=rng)
    assert_cluster_parity(sc, ctx, g, 50, 4)


def test_batch_equals_alone(sc, ctx):
    specs = graphgen.batch_specs(count=12, seed=11, lg_lo=8, lg_hi=13)
    graphs = [s.make() for s in specs]
    ks = [s.k for s in specs]
    devs = [dev(sc, g) for g in graphs]
    parts, sts = sc.partition_batch(ctx, devs, ks)
    for g, d, k, p, st in zip(graphs, devs, ks, parts, sts):
        want_part, want = oracle.partition(g, k)
        assert np.array_equal(host(p), want_part), g.name
        assert st["cut"] == want["cut"] and st["moved_c"] == want["moved_c"]


def test_validate(sc, ctx):
    g = graphgen.rmat(10, 4, seed=1)
    assert sc.validate(ctx, dev(sc, g)) == sc.OK
    bad = graphgen.Graph(g.row_ptr, g.col.copy())
    bad.col[0] = (bad.col[0] + 1) % g.n
    assert sc.validate(ctx, dev(sc, bad)) in (sc.ENOTSYM, sc.EINVAL)
    sl = from_edges(3, [(0, 1), (1, 2)])
    sl.col[0] = 0  # a self-loop in row 0
    assert sc.validate(ctx, dev(sc, sl)) == sc.ENOTSYM


def test_empty_graph(sc, ctx):
    """n = 0: every entry point gives the oracle's trivial result (no labels,
    an empty coarse graph, cut 0, the rounds of the stop rules), also inside
    a batch beside a non-empty graph."""
    g = graphgen.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), name="empty")
    for rule in (0, 1):
        want = oracle.cluster(g, 5, 7, rule, 1)
        lab, ncl, rs = sc.cluster(ctx, dev(sc, g), 5, 7, rule, 1)
        assert host(lab).size == 0 and ncl == 0
        assert rs["rounds"] == want.rounds and rs["moved"] == want.moved and rs["visits"] == want.visits
    assert_contract_parity(sc, ctx, g, np.zeros(0, np.int32), 0)
    assert host(sc.initial_partition(ctx, dev(sc, g), 3)).size == 0
    _, rounds, moved, visits = oracle.refine(g, np.zeros(0, np.int32), 2, 0, 8)
    p = torch.zeros(0, dtype=torch.int32, device="cuda")
    _, rs = sc.refine(ctx, dev(sc, g), p, 2, 0, 8)
    assert rs["rounds"] == rounds and rs["moved"] == moved and rs["visits"] == visits
    want_cut, bw = oracle.cut(g, np.zeros(0, np.int32), 3)
    got, gbw = sc.cut(ctx, dev(sc, g), torch.zeros(0, dtype=torch.int32, device="cuda"), 3)
    assert got == want_cut and list(bw) == gbw
    for k in (1, 4):
        assert_partition_parity(sc, ctx, g, k)
    small = graphgen.rmat(10, 4, seed=2)
    parts, sts = sc.partition_batch(ctx, [dev(sc, g), dev(sc, small)], [4, 4])
    for gg, pp, st in zip((g, small), parts, sts):
        want_part, want = oracle.partition(gg, 4)
        assert np.array_equal(host(pp), want_part), gg.name
        assert st["cut"] == want["cut"] and st["rounds_r"] == want["rounds_r"], gg.name


def many_hubs_graph(seed=12, n=40000, hubs=1100, samples=4600):
    """`hubs` nodes of degree > 4096 joined to random leaves, plus random
    leaf-leaf edges; symmetric CSR with ascending rows."""
    rng = np.random.default_rng(seed)
    u = np.concatenate([np.repeat(np.arange(hubs), samples), rng.integers(hubs, n, 60000)])
    v = np.concatenate([rng.integers(hubs, n, hubs * samples), rng.integers(hubs, n, 60000)])
    keep = u != v
    key = np.unique(np.minimum(u, v)[keep].astype(np.int64) * n + np.maximum(u, v)[keep])
    lo, hi = key // n, key % n
    a, b = np.concatenate([lo, hi]), np.concatenate([hi, lo])
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, a + 1, 1)
    return graphgen.Graph(np.cumsum(rp), b.astype(np.int32))


def test_many_hubs_over_many_rounds(sc, ctx):
    """More than 1024 hubs (degree > 4096) clustered for 8 rounds: the hub
    layout is scanned in several blocks of 1024 hubs and kept over the
    rounds; labels, moves and visits equal the oracle's."""
    g = many_hubs_graph()
    assert (np.diff(g.row_ptr)[:1100] > 4096).all()
    before = ctx.path_counters()
    assert_cluster_parity(sc, ctx, g, 300, 8)
    assert ctx.path_counters()["hub_rounds"] - before["hub_rounds"] == 8


@pytest.mark.parametrize("k", [256, 257])
def test_partition_cut_block_widths(sc, ctx, k):
    """The partition's cut reads the blocks from a one-byte copy when k <= 256
    and from the blocks themselves above: both equal the oracle."""
    name, g = mid_graphs()[2]
    assert_partition_parity(sc, ctx, g, k)
