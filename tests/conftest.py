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
    config.addinivalue_line("markers", "slow: long-running case")


@pytest.fixture(scope="session")
def ara_lib():
    """The built C-ABI library's binding (built in-tree first if absent)."""
    from paper_1308_2066_amd import build as b
    if not os.path.exists(b.LIB):
        b.build(verbose=False)
    from paper_1308_2066_amd import ara
    return ara


@pytest.fixture(scope="session")
def gpu_ctx(ara_lib):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ctx = ara_lib.ara_ctx_create(0)
    yield ctx
    torch.cuda.synchronize()
    ara_lib.ara_ctx_destroy(ctx)
