"""A caller can capture qtx_solve_device in a HIP graph of its own (here a
torch.cuda.CUDAGraph on the context's stream), once a first eager call has
sized the context's workspaces.  Every replay, with the outputs poisoned
and other eager library work and synchronisations in between, reproduces
the eager result bit for bit: FP64 and mixed precision with decimated
self-energies, and the mode-space self-energies at eta = 0."""
import numpy as np
import pytest

from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,method", [(_lib.FP64, 0), (_lib.MIXED, 0), (_lib.FP64, 1)],
                         ids=["fp64", "mixed", "modes"])
def test_solve_device_replays_in_a_graph(gpu_lib, prec, method):
    import torch
    wl = W.config0()
    dev = wl.device
    nE = len(wl.E)
    eta = wl.eta if method == 0 else 0.0
    ctx = _lib.context_for(dev, 0)
    ctx.set_option("self_energy_method", method)
    s = torch.cuda.Stream()
    ctx.set_stream(s.cuda_stream)
    E_t = torch.tensor(wl.E, dtype=torch.float64, device="cuda")
    T_t = torch.empty(nE, dtype=torch.float64, device="cuda")
    L_t = torch.empty((nE, 2, dev.N), dtype=torch.float64, device="cuda")
    I_t = torch.zeros(nE * _lib.INFO_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    def solve():
        ctx.solve_device(E_t.data_ptr(), nE, eta, prec, T_t.data_ptr(), L_t.data_ptr(), I_t.data_ptr())

    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        solve()                                  # sizes the workspaces
    s.synchronize()
    T0, L0, I0 = T_t.clone(), L_t.clone(), I_t.clone()
    assert torch.isfinite(T0).all()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        solve()
    torch.cuda.synchronize()

    other_dev = W.small_random_device(5, 4, 8, uniform=False, same_leads=False, pot_mode=W.POT_LINEAR_FE)
    other = _lib.context_for(other_dev, 0)
    E_other = np.linspace(-1.0, 1.0, 9)
    T_other0 = other.solve(E_other, wl.eta, _lib.FP64)[0]
    for k in range(3):
        T_t.fill_(float("nan"))
        L_t.fill_(float("nan"))
        I_t.fill_(0xAB)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(T_t, T0) and torch.equal(L_t, L0) and torch.equal(I_t, I0), f"replay {k}"
        T_other = other.solve(E_other, wl.eta, _lib.FP64)[0]   # eager work between replays
        assert np.array_equal(T_other, T_other0)
    del g
