import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP engine's Python binding; skips when no device is present."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_08606_amd import sadmm_lib
    return sadmm_lib
