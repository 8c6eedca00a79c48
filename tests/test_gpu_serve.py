"""The continuous-batching loop on the GPU: every request's transmission
and densities equal a solo qtx_solve of the same device and energies, bit
for bit, although requests are admitted, batched together and retired at
different times (devices of different N and m share launches).  Both
precisions; the serving workload specifies the mixed solver."""
import numpy as np
import pytest

from paper_1903_00548_amd import _lib, serve
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [_lib.FP64, _lib.MIXED], ids=["fp64", "mixed"])
def test_served_results_equal_solo_solves(gpu_lib, prec):
    rng = np.random.default_rng(5)
    specs = [(31, 6, 8), (32, 14, 20), (33, 4, 64), (34, 9, 48), (35, 3, 96), (36, 2, 128), (37, 1, 16),
             (38, 12, 33)]
    reqs = []
    for k, (seed, N, m) in enumerate(specs):
        dev = W.small_random_device(seed, N, m, uniform=bool(k % 2), same_leads=bool(k % 3),
                                    pot_mode=W.POT_LINEAR_FE, VL=0.0, VR=-0.02 * k)
        E = np.sort(rng.uniform(-1.8, 1.8, int(rng.integers(9, 40))))
        reqs.append(serve.Request(rid=k, t_arrival=0.0, device=dev, E=E))
    backend = serve.QtxBackend(0, eta=1e-6, precision=prec)
    srv = serve.Server(backend, max_active=3, energies_per_step=7)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs) and st["unfinished"] == 0
    assert max(srv.batch_sizes) > 7                      # launches really mixed several requests
    for r in reqs:
        solo = _lib.context_for(r.device, 0)
        T, L, _, _ = solo.solve(r.E, 1e-6, prec)
        assert np.array_equal(r.T, T), r.rid
        assert np.array_equal(r.ldos, L), r.rid
