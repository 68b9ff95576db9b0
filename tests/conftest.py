import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "perf: timing comparison on the GPU, not a parity test "
                                       "(not marked gpu; run with -m perf)")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def fr():
    """The HIP library binding; GPU tests fail loudly if it cannot load."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    import paper_2406_10262_amd as fr_mod
    fr_mod.load()  # raises if the shared library is missing
    return fr_mod
