import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workload parity (minutes)")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound on cuda:0; fails (does not skip) when it is not there."""
    import torch
    import paper_1909_08006_amd as ley
    assert torch.cuda.is_available(), "gpu-marked test run without a visible GPU"
    ley.load()
    return ley
