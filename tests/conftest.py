import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build_oracle(force=False)
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def gctx():
    """One libgdist context on device 0 for the whole GPU session."""
    from paper_2411_11244_amd import gdist
    ctx = gdist.gdist_create(0)
    yield ctx
    gdist.gdist_destroy(ctx)
