"""Full-size parity in the benchmark's launch configuration: the device
results must equal the oracle's, stored as digests by
tests/golden/make_full_size.py (oracle only)."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")))
FIELDS = ("levels", "n_level", "m_level", "rounds_c", "rounds_r", "moved_c", "moved_r", "visits_c", "visits_r",
          "lmax", "W", "U", "threshold", "n_isolated", "ip_cut", "cut", "max_block")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1402_3281_amd as sc

    c = sc.Context(0)
    yield c
    c.close()


def test_config1_full(ctx):
    import paper_1402_3281_amd as sc

    want = GOLD["cluster"][0]
    g = graphgen.config1_graph()
    d = sc.DeviceGraph.from_host(g, rows_sorted=True)
    lab, ncl, rs = sc.cluster(ctx, d, want["U"], want["rounds"], 0, 1)
    assert digest(lab.cpu().numpy()) == want["labels_sha256"]
    assert rs["moved"] == want["moved"] and rs["visits"] == want["visits"]
    cof, cg = sc.contract(ctx, d, lab)
    h = cg.to_host()
    assert digest(cof.cpu().numpy()) == want["coarse_of_sha256"]
    assert digest(h["col"]) == want["coarse_col_sha256"] and digest(h["ew"]) == want["coarse_ew_sha256"]
    assert int(h["ew"].sum()) // 2 == want["cluster_cut"]


@pytest.mark.parametrize("which", [0, 1])
def test_config2_full(ctx, which):
    import paper_1402_3281_amd as sc

    want = GOLD["partition"][which]
    g = graphgen.config2_graphs()[which]
    assert g.name == want["graph"]
    d = sc.DeviceGraph.from_host(g, rows_sorted=True)
    part, st = sc.partition(ctx, d, want["k"], threshold=want["threshold_arg"])
    assert digest(part.cpu().numpy()) == want["part_sha256"]
    for f in FIELDS:
        assert st[f] == want[f], f
    assert st["max_block"] <= st["lmax"]
