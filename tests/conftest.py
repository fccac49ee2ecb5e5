import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded through its C-ABI binding (GPU tests only)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1905_04975_amd import schur

    schur.load()  # raises if the built library is missing
    return schur
