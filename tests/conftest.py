import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0; builds it first only if nothing is built."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_08132_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2306_08132_amd import build as B
        B.build()
    return _lib.Library.get()
