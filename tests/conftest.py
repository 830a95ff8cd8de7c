import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0; fails loudly when it is not there."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_1110_4874_amd import sht
    sht.load()
    return sht


@pytest.fixture(scope="session")
def plan4095(gpu):
    """The benchmark workload's plan (L = 4095, nside = 2048), built once."""
    return gpu.Plan(4095, 2048)
