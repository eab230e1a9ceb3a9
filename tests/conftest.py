import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU statistics")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def rsk_lib():
    """The built HIP library via its binding; on a GPU machine a missing library is an error."""
    from paper_2203_10838_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("librsk.so is not built: run python -m paper_2203_10838_amd.build")
    return _abi.load()


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to a test marked gpu")
    return torch.device("cuda:0")
