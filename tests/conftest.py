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


# Oracle results on sampled energies of the two full-size workloads, computed
# once per session (a process pool on the host cores) and shared by the FP64
# and mixed full-size tests.
CFG1_SAMPLES = 64
CFG2_SAMPLES = 16


@pytest.fixture(scope="session")
def cfg1_oracle():
    import numpy as np
    import oracle_pool
    from paper_1903_00548_amd import workloads as W
    wl = W.config1()
    rng = np.random.default_rng(1234)
    idx = np.unique(np.concatenate([[0, len(wl.E) - 1],
                                    rng.choice(np.arange(1, len(wl.E) - 1), CFG1_SAMPLES - 2, replace=False)]))
    T, L = oracle_pool.solve("config1", wl.E[idx], wl.eta)
    return wl, idx, T, L


@pytest.fixture(scope="session")
def cfg2_oracle():
    """Eight uniform-grid energies and eight within 1 meV of a lead band
    edge, among them the two hardest of that set for the decimation."""
    import numpy as np
    import oracle_pool
    from paper_1903_00548_amd import workloads as W
    edges = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cfg2_band_edge_energies.txt"))
    wl = W.config2(band_edge_energies=edges)
    n_uni = len(wl.E) - len(edges)
    rng = np.random.default_rng(2345)
    fixed = [7, n_uni - 100, n_uni + 11, n_uni + 150, n_uni + 250, len(wl.E) - 2]
    uni = rng.choice(np.setdiff1d(np.arange(n_uni), fixed), 6, replace=False)
    edge = rng.choice(np.setdiff1d(np.arange(n_uni, len(wl.E)), fixed), 4, replace=False)
    idx = np.unique(np.concatenate([fixed, uni, edge]))
    assert len(idx) == CFG2_SAMPLES
    T, L = oracle_pool.solve("config2", wl.E[idx], wl.eta)
    return wl, idx, n_uni, T, L
