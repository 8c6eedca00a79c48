"""Launch-shape autotuning (qtx_autotune): the choice is one of the timed
candidates allowed by the kernels' occupancy, later solves use it, and
the launch shape never changes a result."""
import numpy as np
import pytest

from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,N", [(8, 16), (32, 40), (64, 24), (128, 10)])
def test_autotune_picks_a_timed_candidate_and_keeps_results(gpu_lib, m, N):
    dev = W.small_random_device(61 + m, N, m, uniform=True, same_leads=True, pot_mode=W.POT_LINEAR_FE)
    E = np.linspace(-1.5, 1.5, 1024)
    ctx = _lib.context_for(dev, 0)
    T0, L0, _, _ = ctx.solve(E, 1e-6, _lib.FP64)
    wg, times = ctx.autotune(E, 1e-6, _lib.FP64)
    print(f"m={m}: chose {wg} workgroups per CU; ms per candidate {np.round(times, 2).tolist()}")
    assert 1 <= wg <= 4 and times[wg - 1] > 0
    assert times[wg - 1] == min(t for t in times if t > 0)
    assert times[0] > 0 and times[1] > 0          # every block size runs two workgroups per CU
    T1, L1, _, _ = ctx.solve(E, 1e-6, _lib.FP64)
    assert np.array_equal(T0, T1) and np.array_equal(L0, L1)


def test_autotune_errors(gpu_lib):
    ctx = _lib.Context(0)
    with pytest.raises(_lib.QtxError) as ei:
        ctx.autotune(np.zeros(4), 1e-6)
    assert ei.value.status == _lib.ESTATE
    ctx2 = _lib.context_for(W.config0().device, 0)
    with pytest.raises(_lib.QtxError) as ei:
        ctx2.autotune(np.zeros(0), 1e-6)
    assert ei.value.status == _lib.EINVAL
