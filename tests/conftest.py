import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    """Build the generator and oracle shared libraries once (gcc, seconds)."""
    import graphgen
    import oracle

    if not os.path.exists(os.path.join(ROOT, "graphgen", "libgraphgen.so")):
        graphgen.build()
    oracle.build(force=False)  # rebuilt when a source is newer than the library
    yield
