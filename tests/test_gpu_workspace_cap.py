"""The option sweep_workspace_bytes caps the resident workgroups of the
sweeps.  With room for only a few workgroups:
- the single-problem solve (FP64 and mixed) gives the same results bit for
  bit as the full grid;
- the batched solve does too;
- the density-matrix blocks agree to rounding, since their per-workgroup
  sums are grouped differently.
A cap below one workgroup's workspace returns QTX_ENOMEM and leaves the
context usable."""
import numpy as np
import pytest

from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu

ETA = 1e-6


def _padded(m):
    return ((m + 15) // 16) * 16 if m <= 64 else (96 if m <= 96 else 128)


def _ws_bytes(N, m, mixed=False, dm=False):
    """Per-workgroup sweep workspace: [X | z] for every slab plus the
    back-substitution buffer(s) in FP64; the mixed sweep's FP32 factors,
    correction columns and FP64 solution."""
    M = _padded(m)
    MM = M * M
    big = 2 * M * (M + 1) * (8 if mixed else 16) if M > 64 else 0
    if not mixed:
        return (N + (2 if dm else 1)) * 2 * MM * 16 + big
    return ((N + 1) * 2 * MM + N * MM + N * 2 * MM + 2 * MM) * 8 + N * 2 * MM * 16 + big


def test_capped_grid_same_results(gpu_lib):
    wl = W.config0()
    dev = wl.device
    E = wl.E
    ctx = _lib.context_for(dev, 0)
    full = {p: ctx.solve(E, ETA, p)[:2] for p in (_lib.FP64, _lib.MIXED)}
    wL = np.linspace(0.3, 1.0, len(E))
    wR = np.linspace(1.0, 0.2, len(E))
    rd0, ro0 = ctx.density_matrix(E, wL, wR, ETA)[:2]
    for prec, mixed in ((_lib.FP64, False), (_lib.MIXED, True)):
        ctx.set_option("sweep_workspace_bytes", 3.5 * _ws_bytes(dev.N, dev.m, mixed))   # three workgroups
        T, L = ctx.solve(E, ETA, prec)[:2]
        assert np.array_equal(T, full[prec][0]) and np.array_equal(L, full[prec][1]), prec
    ctx.set_option("sweep_workspace_bytes", 2.5 * _ws_bytes(dev.N, dev.m, dm=True))      # two workgroups
    rd, ro = ctx.density_matrix(E, wL, wR, ETA)[:2]
    scale = max(1.0, np.abs(rd0).max())
    assert np.abs(rd - rd0).max() <= 1e-13 * scale and np.abs(ro - ro0).max() <= 1e-13 * scale

    ctx.set_option("sweep_workspace_bytes", 0.5 * _ws_bytes(dev.N, dev.m))
    with pytest.raises(_lib.QtxError) as ei:
        ctx.solve(E, ETA, _lib.FP64)
    assert ei.value.status == _lib.ENOMEM
    assert b"sweep_workspace_bytes" in ctx.lib.qtx_last_error(ctx.h)
    ctx.set_option("sweep_workspace_bytes", 160.0 * (1 << 30))
    T, L = ctx.solve(E, ETA, _lib.FP64)[:2]
    assert np.array_equal(T, full[_lib.FP64][0]) and np.array_equal(L, full[_lib.FP64][1])


def test_capped_batch_same_results(gpu_lib):
    devs = [W.small_random_device(s, N, m, uniform=False, same_leads=False, pot_mode=W.POT_LINEAR_FE)
            for s, N, m in ((21, 7, 12), (22, 4, 40), (23, 9, 12))]
    grids = [np.linspace(-1.0, 1.0, n) for n in (11, 6, 9)]
    ref = _lib.Context(0)
    rp = [_lib.fill(ref.problem(), d) for d in devs]
    Tr, Lr, _ = _lib.solve_batch(ref, rp, grids, ETA)
    ctx = _lib.Context(0)
    ctx.set_option("sweep_workspace_bytes", 2.5 * max(_ws_bytes(d.N, d.m) for d in devs))
    probs = [_lib.fill(ctx.problem(), d) for d in devs]
    for _ in range(2):                                # captured graph, then its replay
        Ts, Ls, _ = _lib.solve_batch(ctx, probs, grids, ETA)
        for k in range(len(devs)):
            assert np.array_equal(Ts[k], Tr[k]) and np.array_equal(Ls[k], Lr[k]), k


def test_out_of_memory_lowers_the_budget(gpu_lib):
    """With the budget at its maximum, the full grid of a long m = 128 device
    asks for more workspace than the device has. The first allocation runs
    out of memory, and the context halves its budget until the workspace
    fits. The results equal those of a context with an explicit smaller
    budget bit for bit. That context is solved first and closed, so the two
    workspaces never coexist. The lowered budget stays for the next call."""
    import torch
    N, m, nE = 1400, 128, 512
    lead = W.random_lead(np.random.default_rng(71), m)
    dev = W.Device(N=N, m=m, lead_L=lead, lead_R=lead, V=np.zeros(N), pot_mode=W.POT_DIAG)
    E = np.linspace(-1.2, 1.2, nE)
    ws = _ws_bytes(N, m)
    total = torch.cuda.get_device_properties(0).total_memory
    assert min(nE, 512) * ws > total                  # the full grid cannot be allocated

    ref = _lib.context_for(dev, 0)
    ref.set_option("sweep_workspace_bytes", 128.5 * ws)   # 128 workgroups
    Tr, Lr = ref.solve(E, ETA, _lib.FP64)[:2]
    ref.close()
    torch.cuda.synchronize()

    ctx = _lib.context_for(dev, 0)
    ctx.set_option("sweep_workspace_bytes", 1e13)
    T, L = ctx.solve(E, ETA, _lib.FP64)[:2]
    assert np.array_equal(T, Tr) and np.array_equal(L, Lr)
    T2 = ctx.solve(E[:64], ETA, _lib.FP64)[0]           # the lowered budget is kept
    assert np.array_equal(T2, Tr[:64])
    ctx.close()
