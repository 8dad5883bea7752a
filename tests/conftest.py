import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def bfx():
    """The HIP library on cuda:0 (the import itself fails if libbfx.so is missing)."""
    import torch
    import paper_1904_06376_amd as bfx_mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return bfx_mod


def pytest_collection_modifyitems(config, items):
    # print the test id before each GPU test so a box-level failure names its case
    for it in items:
        if it.get_closest_marker("gpu") is not None:
            it.user_properties.append(("gpu", True))


@pytest.fixture(autouse=True)
def _announce_gpu(request):
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    yield
