"""Shared test setup: repo root on sys.path, the `gpu` marker, and a built library."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")


@pytest.fixture(scope="session")
def lib():
    """The HIP library, built in-tree if it is not there yet."""
    from paper_2508_05400_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        from paper_2508_05400_amd.build import build
        build()
    return _binding.load()


@pytest.fixture(scope="session")
def cuda():
    """torch with a visible GPU (GPU tests fail loudly without one)."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return torch
