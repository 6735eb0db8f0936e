import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle pins (still part of the CPU suite)")


@pytest.fixture(scope="session")
def ct():
    """The product binding (loads the built libct.so)."""
    import paper_2511_11514_amd as ct_mod
    return ct_mod
