import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    # load what is built; build only when nothing is (hipcc cross-compiles gfx950 without a GPU)
    lib = os.path.join(ROOT, "paper_2602_14493_amd", "libgmr.so")
    if not os.path.exists(lib):
        from paper_2602_14493_amd import build as _build
        _build.build()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not gpu_available():
        pytest.fail("GPU test selected but no GPU is visible")
    import paper_2602_14493_amd as gmr
    return gmr
