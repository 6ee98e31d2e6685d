import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU case")


@pytest.fixture(scope="session")
def mfa():
    """(binding module, context on device 0) for GPU tests."""
    import torch

    from paper_2204_11762_amd import binding as b
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = b.mfa_create(0)
    yield b, ctx
    b.mfa_destroy(ctx)
