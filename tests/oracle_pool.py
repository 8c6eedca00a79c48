"""The FP64 oracle on sampled energies of the full-size workloads, one
energy per task over a pool of host processes (the oracle is serial per
energy: tens of seconds at N = 400, m = 128).  Workers rebuild the seeded
device from its workloads builder, so nothing but the builder's name and
the energies crosses the process boundary.  Test infrastructure only."""
import multiprocessing as mp
import os

import numpy as np

_DEV = {}


def _device(builder):
    if builder not in _DEV:
        from paper_1903_00548_amd import workloads
        _DEV[builder] = getattr(workloads, builder)().device
    return _DEV[builder]


def _solve_one(args):
    builder, E, eta = args
    import oracle
    T, nL, nR = oracle.solve_energy(_device(builder), float(E), eta)
    return T, nL, nR


def solve(builder, energies, eta, workers=None):
    """T (nE,) and ldos (nE, 2, N) of workloads.<builder>()'s device."""
    energies = np.asarray(energies, dtype=np.float64)
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0)), len(energies)))
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"                       # one BLAS thread per worker
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            out = pool.map(_solve_one, [(builder, E, eta) for E in energies], chunksize=1)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    T = np.array([o[0] for o in out])
    ldos = np.stack([np.stack([o[1], o[2]]) for o in out])
    return T, ldos
