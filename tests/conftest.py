import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def engine():
    """Engine on cuda:0; GPU tests only (fails loudly if the library is missing)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_08968_amd as dx
    return dx.Engine(0)
