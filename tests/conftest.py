import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical check")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    # GPU tests fail loudly (not skip) when selected explicitly with -m gpu on a
    # machine without a GPU; when not selected they are deselected by -m.
    pass


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; GPU tests require it."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_2602_14975_amd import nnp
    nnp.lib()  # raises if the shared library is missing
    return nnp
