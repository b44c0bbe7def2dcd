"""The allocation-free cut entry point against sclap_cut on the same inputs,
through the C ABI: two calls in a row, the second on a smaller graph (the
fixed scratch keeps the first call's partial sums), then a weighted graph."""
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


def run_both(sc, ctx, g, part, k):
    d = sc.DeviceGraph.from_host(g)
    p = torch.from_numpy(part).cuda()
    want_cut, want_bw = sc.cut(ctx, d, p, k)
    cut = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    bw = torch.full((k,), -1, dtype=torch.int64, device="cuda")
    sc.cut_noalloc(d, p, k, cut, bw)
    torch.cuda.synchronize()
    got_cut, got_bw = int(cut.cpu()[0]), bw.cpu().numpy().tolist()
    ocut, obw = oracle.cut(g, part, k)
    assert got_cut == want_cut == ocut
    assert got_bw == list(want_bw) == [int(x) for x in obw]
    # the cut alone (no block weights)
    cut2 = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    sc.cut_noalloc(d, p, k, cut2, None)
    torch.cuda.synchronize()
    assert int(cut2.cpu()[0]) == ocut


def test_noalloc_cut_matches_cut_twice(sc):
    with sc.Context(0) as ctx:
        big = graphgen.rmat(19, 16, seed=2)          # about 7k cut workgroups: most of the scratch
        rng = np.random.default_rng(3)
        run_both(sc, ctx, big, rng.integers(0, 16, size=big.n).astype(np.int32), 16)
        small = graphgen.rgg(3000, 8.0, seed=5)      # fewer partial sums than the call before
        run_both(sc, ctx, small, rng.integers(0, 4, size=small.n).astype(np.int32), 4)
        g = graphgen.rmat(10, 8, seed=7)
        w = graphgen.Graph(g.row_ptr, g.col, ew=(1 + (g.col % 5)).astype(np.int32),
                           nw=rng.integers(0, 9, size=g.n).astype(np.int64))
        # symmetric edge weights: weight of {u, v} from min and max of the pair
        u = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        w.ew = (1 + (np.minimum(u, g.col) * 7 + np.maximum(u, g.col)) % 5).astype(np.int32)
        run_both(sc, ctx, w, rng.integers(0, 3, size=g.n).astype(np.int32), 3)


def test_noalloc_rejects_k_beyond_limit(sc):
    g = graphgen.rmat(8, 4, seed=1)
    d = sc.DeviceGraph.from_host(g)
    p = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    cut = torch.zeros(1, dtype=torch.int64, device="cuda")
    bw = torch.zeros(5000, dtype=torch.int64, device="cuda")
    with pytest.raises(sc.SclapError) as e:
        sc.cut_noalloc(d, p, 5000, cut, bw)
    assert e.value.code == sc.EINVAL
    sc.cut_noalloc(d, p, 5000, cut, None)   # the cut alone has no k limit
    torch.cuda.synchronize()
    assert int(cut.cpu()[0]) == 0
