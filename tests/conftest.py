import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running GPU case at full workload size")


def _gpu_available() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip-free guard: GPU tests must fail loudly, not skip, when the device or
    the HIP library is missing on a machine with a GPU."""
    if not _gpu_available():
        pytest.fail("GPU test selected but torch sees no GPU")
    import paper_1312_6182_amd as g
    g.load()  # raises if libgpspca.so is missing
    return g
