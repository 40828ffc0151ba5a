import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; GPU tests only."""
    import paper_1110_3105_amd as rs
    if not rs.device_available():
        pytest.fail("no HIP device visible: GPU tests must run on an MI355X")
    return rs
