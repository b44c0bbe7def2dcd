"""Contraction element by element against the oracle at the sizes where the
coarse keys are 30 to 34 bits wide (coarse node counts 2^15 to 2^17), on
unit and weighted levels, and the multilevel partitions of the two served
random geometric graphs whose contractions sort such keys in arrays of
1024 < n <= 2^20 items (the radix sort's merge-sort range)."""
import numpy as np
import pytest

import graphgen
import oracle

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


def weighted(g):
    u = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    v = g.col.astype(np.int64)
    ew = (1 + (np.minimum(u, v) * 31 + np.maximum(u, v)) % 7).astype(np.int32)
    nw = (1 + np.arange(g.n) % 3).astype(np.int64)
    return graphgen.Graph(g.row_ptr, g.col, ew=ew, nw=nw, name=g.name + "-w")


@pytest.mark.parametrize("nc_target", [20000, 40000, 70000])
@pytest.mark.parametrize("weighted_level", [False, True])
def test_contract_at_key_widths(sc, ctx, nc_target, weighted_level):
    g = graphgen.rgg(200000, 8.0, seed=11)
    if weighted_level:
        g = weighted(g)
    # clusters of consecutive ids (ids are spatially ordered in the RGG): many
    # coarse edges, coarse node counts around nc_target
    size = max(1, g.n // nc_target)
    labels = (np.arange(g.n) // size * size).astype(np.int32)
    want = oracle.contract(g, labels)
    d = sc.DeviceGraph.from_host(g)
    cof, cg = sc.contract(ctx, d, torch.from_numpy(labels).cuda())
    got = cg.to_host()
    torch.cuda.synchronize()
    assert want.n == len(set(labels.tolist()))
    assert np.array_equal(cof.cpu().numpy(), want.coarse_of)
    assert np.array_equal(got["row_ptr"], want.row_ptr)
    assert np.array_equal(got["col"], want.col)
    assert np.array_equal(got["ew"], want.ew)
    assert np.array_equal(got["nw"], want.nw)
    cg.close()


@pytest.mark.parametrize("index", [45, 61])
def test_served_rgg_partition(sc, ctx, index):
    spec = graphgen.serve_specs(count=index + 1, seed=4)[index]
    g = spec.make()
    print(f"partition of served graph {index}: {spec.kind} n={g.n} k={spec.k}", flush=True)
    want_part, want = oracle.partition(g, spec.k)
    part, st = sc.partition(ctx, sc.DeviceGraph.from_host(g, rows_sorted=True), spec.k)
    assert np.array_equal(part.cpu().numpy(), want_part)
    assert st["cut"] == want["cut"] and st["levels"] == want["levels"]
    assert st["n_level"] == want["n_level"] and st["m_level"] == want["m_level"]
