"""The degree bins' bounds and their autotuner: every admissible set of
bounds gives the oracle's result (the bounds only choose which kernel rates
a node), alone and in fused batches; the autotuner keeps an admissible set."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOUNDS = [[64, 128, 512, 1024], [32, 64, 128, 512], [64, 128, 256, 1024], [32, 128, 512, 512],
          [64, 64, 128, 512], [32, 32, 32, 32], [64, 128, 512, 2048], [32, 64, 256, 2048]]


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


@pytest.mark.parametrize("hi", BOUNDS, ids=lambda h: "-".join(map(str, h)))
def test_bounds_keep_results(sc, ctx, hi):
    ctx.set_bin_bounds(hi)
    try:
        for g, k in ((graphgen.rmat(15, 16, seed=2), 8), (graphgen.rgg(1 << 14, 9.0, seed=5), 4)):
            print(f"bounds {hi} {g.name}", flush=True)
            d = sc.DeviceGraph.from_host(g)
            lab, nc, rs = sc.cluster(ctx, d, 200, 6, 0, 1)
            want = oracle.cluster(g, 200, 6, 0, 1)
            assert np.array_equal(lab.cpu().numpy(), want.labels)
            assert rs["moved"] == want.moved and rs["visits"] == want.visits
            part, st = sc.partition(ctx, d, k)
            wp, wst = oracle.partition(g, k)
            assert np.array_equal(part.cpu().numpy(), wp) and st["cut"] == wst["cut"]
    finally:
        ctx.set_bin_bounds([64, 128, 512, 1024])


def test_bounds_in_a_fused_batch(sc, ctx):
    specs = graphgen.batch_specs(count=12, seed=77, lg_lo=10, lg_hi=14)
    graphs = [s.make() for s in specs]
    devs = [sc.DeviceGraph.from_host(g) for g in graphs]
    ctx.set_bin_bounds([32, 64, 256, 512])
    try:
        parts, sts = sc.partition_batch(ctx, devs, [s.k for s in specs])
    finally:
        ctx.set_bin_bounds([64, 128, 512, 1024])
    for g, s, p, st in zip(graphs, specs, parts, sts):
        wp, wst = oracle.partition(g, s.k)
        assert np.array_equal(p.cpu().numpy(), wp), g.name
        assert st["cut"] == wst["cut"]


def test_invalid_bounds_rejected(sc, ctx):
    for hi in ([16, 64, 128, 512], [64, 32, 128, 512], [64, 128, 1024, 1024], [64, 128, 512, 4096]):
        with pytest.raises(sc.SclapError):
            ctx.set_bin_bounds(hi)
    assert ctx.bin_bounds() == [64, 128, 512, 1024]


def test_autotune_keeps_admissible_bounds(sc):
    g = graphgen.rmat(16, 16, seed=9)
    d = sc.DeviceGraph.from_host(g)
    with sc.Context(0) as c:
        r = c.autotune(d, 300, rounds=2)
        print(r, flush=True)
        hi = r["bounds"]
        assert 32 <= hi[0] <= 64 and hi[0] <= hi[1] <= 128 and hi[1] <= hi[2] <= 512 and hi[2] <= hi[3] <= 2048
        assert c.bin_bounds() == hi
        assert 0 < r["ms"] <= r["default_ms"]
        part, st = sc.partition(c, d, 16)
        wp, wst = oracle.partition(g, 16)
        assert np.array_equal(part.cpu().numpy(), wp)
