"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only bounds call matches the closed forms."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sclap.h")
LIB = os.path.join(ROOT, "paper_1402_3281_amd", "libsclap.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sclap_[a-z_]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = declared_functions()
    for want in ("sclap_create", "sclap_bounds", "sclap_cluster", "sclap_contract", "sclap_refine", "sclap_cut",
                 "sclap_partition", "sclap_partition_batch", "sclap_server_create", "sclap_server_submit"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsclap.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsclap.so not built")
def test_binding_signatures_cover_header():
    import paper_1402_3281_amd as sc

    assert set(declared_functions()) == set(sc.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsclap.so not built")
def test_bounds_golden_via_abi():
    import paper_1402_3281_amd as sc

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "bounds.json")))
    for case in gold["cases"]:
        assert sc.bounds(case["total_w"], case["max_w"], case["k"]) == (case["lmax"], case["W"], case["U"])
    with pytest.raises(sc.SclapError):
        sc.bounds(10, 1, 0)
    with pytest.raises(sc.SclapError):
        sc.bounds(10, 1, 2, eps=(1, 0))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsclap.so not built")
def test_server_footprint_bounds():
    """The bytes a server charges for a job cover what the job holds on the
    device at once: the input copy, two weighted hierarchy copies, the LP
    state with refinement's block connections, the per-node and per-entry
    scratch of the fused rounds (degree bins 9 x (4 + 8) B, hub rows 16 B,
    rated list and movers 12 B, contended keys and their buffers 36 B per
    node, byte copies of the blocks; staged hub pairs, bounded here by
    16 B x 1.5 per entry; tile rows) and a contraction's temporaries (the
    cross keys as emitted, room for every entry at 8 B, and four 8 B arrays
    per undirected edge)."""
    import paper_1402_3281_amd as sc

    for n, m, k, ew, nwb in ((1 << 10, 16 << 10, 2, False, 0), (1 << 20, 32 << 20, 64, False, 0),
                             (1 << 16, 1 << 20, 128, True, 8), (5, 0, 3, False, 4), (0, 0, 1, False, 0)):
        inp, fp = sc.server_footprint(n, m, k, ew, nwb)
        assert inp == 8 * (n + 1) + 4 * m + (4 * m if ew else 0) + nwb * n
        hierarchy = 2 * (8 * (n + 1) + 8 * m + 12 * n)
        conn = 4 * n * k if k <= 64 else 0
        round_scratch = n * (9 * 12 + 16 + 12 + 36) + int(1.5 * 16 * m)
        contraction = 8 * m + 4 * 8 * (m // 2)
        assert fp >= inp + hierarchy + 48 * n + conn + round_scratch + contraction, (n, m, k)
    # monotone in the graph size and in k up to the block-connection limit
    a = sc.server_footprint(1000, 8000, 4)[1]
    assert sc.server_footprint(2000, 8000, 4)[1] > a and sc.server_footprint(1000, 16000, 4)[1] > a
    assert sc.server_footprint(1000, 8000, 8)[1] > a
    with pytest.raises(sc.SclapError):
        sc.server_footprint(10, 10, 0)
