"""Shared pytest configuration.

Tests marked ``gpu`` run the HIP library on an MI355X through its C ABI;
everything else runs on the CPU (oracle pins, input recipes, host-side
argument validation, symbol exports).
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X; calls the HIP library through its C ABI")


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding, with a device present (fails loudly otherwise)."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_2608_11882_amd as hc
    hc.load()  # raises if the HIP library is not built
    return hc


@pytest.fixture
def one_step(gpu):
    """One step per pass for the duration of a test: the single-step
    kernels (the library takes two steps per pass by default)."""
    saved = gpu.get_time_block()
    gpu.set_time_block(1)
    yield gpu
    gpu.set_time_block(saved)


@pytest.fixture(params=[1, 2], ids=["one_step", "two_steps"])
def time_block(request, gpu):
    """Run a test with one, then two steps per pass (restored afterwards)."""
    saved = gpu.get_time_block()
    gpu.set_time_block(request.param)
    yield request.param
    gpu.set_time_block(saved)
