import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """The oracle is C; build it once per session if its libraries are absent."""
    here = os.path.join(ROOT, "oracle")
    libs = [os.path.join(here, n) for n in ("liborc_pt2.so", "liborc_fci.so")]
    if not all(os.path.exists(p) for p in libs):
        from oracle import build
        build.build()
    yield
