import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def ctx():
    """One library context on cuda:0 for the whole GPU session."""
    import torch
    from paper_2306_03651_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    binding.lib()   # raises if the HIP library is not built: no fallback
    c = binding.centra_create(0, 0)
    yield c
    torch.cuda.synchronize()
    binding.centra_destroy(c)
