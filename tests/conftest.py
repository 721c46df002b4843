import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle case")


@pytest.fixture(scope="session")
def gpu_lib():
    """The GPU library, loaded through its C-ABI binding. Fails (never skips) on a
    GPU machine where the library is missing."""
    import paper_2308_08447_amd as pkg
    return pkg.load()
