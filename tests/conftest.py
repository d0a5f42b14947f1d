import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests run only where a GPU is present; on a CPU-only machine they are skipped
    # with a reason (select them with -m gpu on a machine with an MI355X).
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this process")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def rlbm_lib():
    """The built HIP library (built in place if it is missing)."""
    from paper_1909_04502_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    from paper_1909_04502_amd import rlbm
    return rlbm.lib()
