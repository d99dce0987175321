import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library; GPU tests fail loudly if it is missing."""
    from paper_2508_04172_amd import rbfl
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    return rbfl.load()
