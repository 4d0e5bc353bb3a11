import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X / gfx950) and the HIP library")
    config.addinivalue_line("markers", "slow: long-running (full-size workloads)")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle.build import ensure_built
    ensure_built()
    import oracle
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The product library on cuda:0; builds libeik.so only if it is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_2103_05694_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    import paper_2103_05694_amd as eik
    eik.api._lib.load()
    return eik
