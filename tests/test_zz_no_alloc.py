"""The no-allocation solve (qtx_solve_device_noalloc) against the ordinary
device-pointer solve (qtx_solve_device) through the C ABI: the same
kernels run on the same energies, only the buffers come from the
library's fixed device scratch, so T, the slab densities and the
diagnostics must agree bit for bit.  Two calls in a row on one context,
the second with a smaller energy grid, in FP64 and in mixed precision;
and a problem too large for the scratch is refused with QTX_ENOMEM."""
import numpy as np
import pytest

from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu


def _solve_pair(ctx, E, eta, prec, N):
    import torch
    E_t = torch.tensor(E, dtype=torch.float64, device="cuda")
    out = []
    for fn in (ctx.solve_device, ctx.solve_device_noalloc):
        T = torch.full((len(E),), float("nan"), dtype=torch.float64, device="cuda")
        L = torch.full((len(E), 2, N), float("nan"), dtype=torch.float64, device="cuda")
        info = torch.zeros((len(E), _lib.INFO_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
        fn(E_t.data_ptr(), len(E), eta, prec, T.data_ptr(), L.data_ptr(), info.data_ptr())
        torch.cuda.synchronize()
        out.append((T.cpu().numpy(), L.cpu().numpy(), info.cpu().numpy().view(_lib.INFO_DTYPE).reshape(-1)))
    return out


def _same(a, b, label):
    (Ta, La, ia), (Tb, Lb, ib) = a, b
    assert np.all(np.isfinite(Ta)) and np.all(np.isfinite(La)), label
    assert np.array_equal(Ta, Tb), f"{label}: T differs, max {np.abs(Ta - Tb).max():.3e}"
    assert np.array_equal(La, Lb), f"{label}: densities differ, max {np.abs(La - Lb).max():.3e}"
    for f in ("dec_iters", "refine_steps", "fell_back_fp64", "flags"):
        assert np.array_equal(ia[f], ib[f]), f"{label}: info.{f} differs"
    assert np.array_equal(ia["resid"], ib["resid"]), f"{label}: info.resid differs"


def _ctx_on_torch_stream(dev):
    import torch
    ctx = _lib.context_for(dev, 0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    return ctx


@pytest.mark.parametrize("prec", [_lib.FP64, _lib.MIXED], ids=["fp64", "mixed"])
def test_noalloc_matches_solve_device_tiny(gpu_lib, prec):
    wl = W.config0()
    ctx = _ctx_on_torch_stream(wl.device)
    a, b = _solve_pair(ctx, wl.E, wl.eta, prec, wl.device.N)
    _same(a, b, "tiny, first call (64 energies)")
    E2 = np.linspace(-2.1, 2.7, 17)
    a, b = _solve_pair(ctx, E2, wl.eta, prec, wl.device.N)
    _same(a, b, "tiny, second call (17 energies)")
    ctx.close()


def test_noalloc_matches_solve_device_headline_fp64(gpu_lib):
    """N = 200, m = 64: the 2048-energy grid runs in several chunks of the
    scratch, then a smaller grid of other energies on the same context."""
    wl = W.config1()
    ctx = _ctx_on_torch_stream(wl.device)
    a, b = _solve_pair(ctx, wl.E, wl.eta, _lib.FP64, wl.device.N)
    _same(a, b, "N=200 m=64, 2048 energies")
    E2 = np.linspace(-1.2, 1.3, 300)
    a, b = _solve_pair(ctx, E2, wl.eta, _lib.FP64, wl.device.N)
    _same(a, b, "N=200 m=64, 300 energies")
    ctx.close()


def test_noalloc_matches_solve_device_headline_mixed(gpu_lib):
    wl = W.config1()
    ctx = _ctx_on_torch_stream(wl.device)
    a, b = _solve_pair(ctx, wl.E[::32], wl.eta, _lib.MIXED, wl.device.N)
    _same(a, b, "N=200 m=64 mixed, 64 energies")
    a, b = _solve_pair(ctx, wl.E[5::97], wl.eta, _lib.MIXED, wl.device.N)
    _same(a, b, "N=200 m=64 mixed, 22 energies")
    ctx.close()


def test_noalloc_refuses_a_problem_beyond_the_scratch(gpu_lib):
    import torch
    rng = np.random.default_rng(5)
    lead = W.random_lead(rng, 128)
    ctx = _lib.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    for side in (_lib.LEFT, _lib.RIGHT):
        ctx.set_lead(side, lead.H00, lead.H01, lead.S00, lead.S01, 0.0)
    ctx.set_device(3000, 128)           # one energy's sweep workspace alone is 1.6 GB
    E = torch.zeros(4, dtype=torch.float64, device="cuda")
    T = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.QtxError) as ei:
        ctx.solve_device_noalloc(E.data_ptr(), 4, 1e-6, _lib.FP64, T.data_ptr())
    assert ei.value.status == _lib.ENOMEM
    assert "no-allocation scratch" in str(ei.value)
    ctx.close()
