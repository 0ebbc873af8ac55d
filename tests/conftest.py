import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: runs HIP kernels on the GPU through the C ABI")


@pytest.fixture(scope="session")
def lib():
    """The built libtsmg.so, on a machine with a GPU (fails loudly otherwise)."""
    import torch
    from paper_1901_00654_amd import tsmg
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return tsmg.load_library()
