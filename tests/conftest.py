import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def gpu_ctx():
    """One library context for the whole GPU session (skips without a device)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU device")
    import paper_2008_03095_amd as P

    ctx = P.Context(device=0)
    yield ctx
    ctx.close()


def announce(msg: str):
    """Names the GPU case about to run (flushed, so a crash log shows it)."""
    print(f"\n[gpu-case] {msg}", flush=True)
