import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(autouse=True)
def _seeded_torch():
    """Every test starts from the same torch generator state (CPU and GPU), so
    inputs drawn with torch are seeded like the numpy ones, whatever ran
    before."""
    try:
        import torch
    except ImportError:
        yield
        return
    torch.manual_seed(20220404)
    yield
