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
