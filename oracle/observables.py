"""Transmission and slab-resolved density of states (oracle, FP64).

Test infrastructure only (see the package docstring).

For ballistic transport the wave-function (QTBM) and Green's-function
routes give the same observables (Sec. "Extended states", last paragraph),
so the oracle uses the Green's-function form with the full broadening of
each contact as injection:

    T(E)   = Re Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H]
    n^L_i  = (1/pi) Re sum_{j in slab i} [G_{:,0} Gamma_L G_{:,0}^H]_jj
    n^R_i  = (1/pi) Re sum_{j in slab i} [G_{:,N-1} Gamma_R G_{:,N-1}^H]_jj

n counts states per eV and per slab with spin degeneracy 2 (the node
density of Sec. "Density" with g = 2/|v| for flux-normalised modes equals
(1/pi) diag(G Gamma G^H); see oracle.qtbm).
"""
from __future__ import annotations

import numpy as np

from .leads import self_energies, broadening
from .device import (potential_weights, assemble, first_block_column,
                     last_block_column, columns_dense, columns_banded,
                     columns_two_pass)


def transmission(G_N0, gamma_L, gamma_R):
    return float(np.real(np.trace(gamma_R @ G_N0 @ gamma_L @ G_N0.conj().T)))


def slab_dos(Gcol, gamma):
    """(1/pi) Re diag(G Gamma G^H), summed within each slab: (N,)."""
    GG = Gcol @ gamma                       # (N, m, m)
    return np.real(np.einsum("nij,nij->n", GG, Gcol.conj())) / np.pi


def _leads_of(dev):
    L, R = dev.lead_L, dev.lead_R
    return ((L.H00, L.H01, L.S00, L.S01, L.V),
            (R.H00, R.H01, R.S00, R.S01, R.V))


def solve_energy(dev, E, eta, method="right", sigma=None):
    """T, n^L (N,), n^R (N,) at one energy for a device object with the
    attributes of a transport problem (N, m, lead_L, lead_R, V, pot_mode
    and blocks())."""
    z = E + 1j * eta
    lead_L, lead_R = _leads_of(dev)
    if sigma is None:
        sigL, sigR = self_energies(z, lead_L, lead_R, eta)
    else:
        sigL, sigR = sigma
    Hd, Hu, Sd, Su = dev.blocks()
    Vd, Vu = potential_weights(dev.V, lead_L[4], lead_R[4], dev.pot_mode)
    Ad, Au, Al = assemble(z, Hd, Hu, Sd, Su, Vd, Vu)
    Ad = Ad.copy()
    Ad[0] = Ad[0] - sigL
    Ad[-1] = Ad[-1] - sigR
    if method == "right":
        G0 = first_block_column(Ad, Au, Al)
        GN = last_block_column(Ad, Au, Al)
    elif method == "two_pass":
        G0, GN = columns_two_pass(Ad, Au, Al)
    elif method == "dense":
        G0, GN = columns_dense(Ad, Au, Al)
    elif method == "banded":
        G0, GN = columns_banded(Ad, Au, Al)
    else:
        raise ValueError(method)
    gL = broadening(sigL)
    gR = broadening(sigR)
    T = transmission(G0[-1], gL, gR)
    nL = slab_dos(G0, gL)
    nR = slab_dos(GN, gR)
    return T, nL, nR


def solve_device(dev, energies, eta, method="right"):
    """T (nE,) and ldos (nE, 2, N) over an energy grid."""
    energies = np.asarray(energies, dtype=np.float64)
    nE = energies.shape[0]
    T = np.empty(nE)
    ldos = np.empty((nE, 2, dev.N))
    for k, E in enumerate(energies):
        T[k], ldos[k, 0], ldos[k, 1] = solve_energy(dev, float(E), eta, method)
    return T, ldos
