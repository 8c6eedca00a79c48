import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded once per session; fails loudly if absent.

    PyTorch is initialised first, as in the benchmark and in production
    use (PyTorch owns device memory and streams): the library then binds
    to the HIP runtime that torch loaded, and torch tensors and streams
    can be handed to it."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    from paper_1903_00548_amd import _lib
    return _lib.load()
