import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def engine():
    """One engine on cuda:0 for the whole GPU session (fails loudly without the library)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2607_17571_amd import wg

    eng = wg.Engine(0)
    yield eng
    eng.close()
