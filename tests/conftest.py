import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X); parity and device tests")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """The loaded GPU library; fails loudly if the HIP extension is missing."""
    if not _gpu_available():
        pytest.skip("no HIP device")
    import paper_1706_02740_amd as sftlib
    sftlib.require_device()
    return sftlib
