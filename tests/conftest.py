import os
import sys

import pytest

# every workspace the library allocates starts as NaN bytes in the tests, so a
# kernel that reads scratch it never wrote fails instead of reading zeros
os.environ.setdefault("RTE_POISON_WORKSPACE", "1")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Device handle for GPU tests; fails loudly (not skip) when the library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2306_05789_amd import rte
    rte.load()  # raises if the HIP library is not built
    return torch.device("cuda:0")
