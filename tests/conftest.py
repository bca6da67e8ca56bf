import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: test taking more than ~20 s on the CPU or minutes on the GPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The native library, loaded for GPU tests; fails loudly if unavailable."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2512_01257_amd import native

    return native
