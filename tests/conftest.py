import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def isr_ctx():
    """One library context for the whole GPU session."""
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2407_20731_amd import isr
    ctx = isr.Context()
    yield ctx
    ctx.close()
