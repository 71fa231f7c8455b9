import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; skips if no GPU is present."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7285_amd import binding
    return binding.load()
