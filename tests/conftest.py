import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libdna.so")


@pytest.fixture(scope="session")
def dna():
    """The HIP binding; GPU tests fail loudly (not skip) when it cannot load."""
    from paper_1301_3389_amd import dna as binding
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return binding
