"""Seeded small devices shared by the FP64 and mixed-precision GPU parity
tests; the oracle result of each case is computed once per session."""
import functools

import numpy as np

import oracle
from paper_1903_00548_amd import workloads as W

ETA = 1e-6

# seed, N, m, uniform device, identical leads, potential mode
CASES = [
    (1, 5, 4, True, True, W.POT_LINEAR_FE),
    (2, 9, 6, False, False, W.POT_LINEAR_FE),
    (3, 1, 16, False, False, W.POT_DIAG),          # a single slab: both contacts on one block
    (4, 2, 16, True, False, W.POT_LINEAR_FE),
    (5, 33, 20, False, True, W.POT_DIAG),          # ragged m (padded to 32), more slabs than tiles
    (6, 17, 48, True, True, W.POT_LINEAR_FE),
    (7, 12, 64, False, False, W.POT_LINEAR_FE),
    (8, 3, 1, True, True, W.POT_DIAG),             # one-band chain
    (9, 4, 80, False, False, W.POT_LINEAR_FE),     # padded to 96: working matrix outside LDS
    (10, 6, 96, True, True, W.POT_DIAG),
    (11, 3, 128, False, True, W.POT_LINEAR_FE),
    (12, 2, 100, True, False, W.POT_DIAG),         # padded to 128
]


def device(seed, N, m, uniform, same, mode):
    return W.small_random_device(seed, N, m, uniform=uniform, same_leads=same, pot_mode=mode,
                                 VL=0.04 * (seed % 3), VR=-0.03 * (seed % 2))


def energies():
    return np.linspace(-2.0, 2.0, 23)


@functools.lru_cache(maxsize=None)
def reference(seed, N, m, uniform, same, mode):
    """(T, ldos) of the oracle for one case."""
    return oracle.solve_device(device(seed, N, m, uniform, same, mode), energies(), ETA)
