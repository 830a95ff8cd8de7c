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


def _log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


@pytest.fixture(scope="session")
def plan4095_bf(gpu):
    """The benchmark workload's butterfly plan (L = 4095, nside = 2048,
    eps = 1e-12, FP32 and transposed copies), from the plan cache or built
    once per session (about two minutes on 16 host cores)."""
    _log("plan4095_bf: L=4095 nside=2048 eps=1e-12 (cache or build)")
    p = gpu.cached_plan(4095, 2048, 1e-12, store_fp32=True, store_transpose=True, log=_log)
    _log(f"plan4095_bf: ready, depth histogram {p.info()['bf_depth_hist'][:6]}")
    return p


@pytest.fixture(scope="session")
def plan2047_bf(gpu):
    """The 16-map workload's butterfly plan (L = 2047, nside = 1024,
    eps = 1e-12, FP32 and transposed copies)."""
    _log("plan2047_bf: L=2047 nside=1024 eps=1e-12 (cache or build)")
    p = gpu.cached_plan(2047, 1024, 1e-12, store_fp32=True, store_transpose=True, log=_log)
    _log(f"plan2047_bf: ready, depth histogram {p.info()['bf_depth_hist'][:6]}")
    return p
