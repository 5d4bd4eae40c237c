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
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.get()


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def xtr():
    """The product binding, on a GPU.  GPU tests fail (not skip) when the
    native library is missing: the HIP path must be the one that runs."""
    if not _gpu_available():
        pytest.skip("no GPU in this process")
    import paper_2605_13864_amd as x
    x.load()          # raises if libxtr.so is missing or does not load
    return x
