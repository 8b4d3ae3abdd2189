import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded for GPU tests.  On a machine without a GPU
    the GPU tests are skipped; with a GPU the library must load (a missing
    extension is an error, never a fallback)."""
    if not _gpu_present():
        pytest.skip("no GPU visible")
    import paper_1802_07525_amd as lbm
    lbm.load()  # raises if the built library is missing
    return lbm
