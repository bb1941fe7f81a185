import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def dev():
    """The HIP device; GPU tests fail (not skip) when it is missing, so that a
    GPU run without a GPU is never reported as green."""
    import torch
    assert torch.cuda.is_available(), "GPU test collected on a host without a GPU"
    return torch.device("cuda:0")
