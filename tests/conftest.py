"""Shared test set-up: repository root on sys.path and the `gpu` marker.

Tests marked `gpu` need an MI355X (gfx950) and the built HIP library; the
rest run on the CPU (oracle pins, host logic, the C ABI's exported symbols
and argument checks)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")


@pytest.fixture(scope="session")
def ref():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def dev():
    """cuda:0 with the built library loaded; GPU tests fail loudly without either."""
    import torch

    import paper_2108_08380_amd as bd
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a ROCm device")
    bd.lib()
    return torch.device("cuda:0")


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()
