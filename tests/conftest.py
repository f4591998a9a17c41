import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# libvc names a failed HIP call or internal check on stderr (failures only)
os.environ.setdefault("VC_DEBUG", "1")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle


@pytest.fixture(scope="session")
def libvc():
    """The built libvc.so (built once if it is not there yet)."""
    from paper_2512_18334_amd import vc
    if not os.path.exists(vc.LIB_PATH):
        from paper_2512_18334_amd import build
        build.build()
    return vc.load()
