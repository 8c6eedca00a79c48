"""Nearest-neighbour density-matrix blocks (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. "Density", eq. density_matrices: the density matrix in the slab
(Bloch-wave) basis is the energy sum, with quadrature weights, occupations
and the density of states of each injected state, of the outer products of
the solution coefficients; the density itself needs only its on-slab and
neighbouring-slab blocks (eq. density_3d_fast).  With the full broadening of
each contact as injection (the Green's-function form of the same
observables, see oracle.observables) the sum over the states of contact X
at one energy is (1/pi) G_{:,X} Gamma_X G_{:,X}^H, so

    rho_ij = sum_e (1/pi) [wL_e G_{i,0}(E_e) Gamma_L G_{j,0}(E_e)^H
                           + wR_e G_{i,N-1}(E_e) Gamma_R G_{j,N-1}(E_e)^H]

for j = i and j = i + 1, where wX_e is the quadrature weight of E_e times
the occupation of contact X.  The paper's n_{i'n'k',ink} (conjugated
coefficient first) is this rho with the two index pairs exchanged.
"""
from __future__ import annotations

import numpy as np

from .leads import self_energies, broadening
from .device import potential_weights, assemble, first_block_column, last_block_column


def energy_blocks(dev, E, eta, sigma=None):
    """G_{:,0}, G_{:,N-1} (N, m, m), Gamma_L, Gamma_R at one energy."""
    L, R = dev.lead_L, dev.lead_R
    lead_L = (L.H00, L.H01, L.S00, L.S01, L.V)
    lead_R = (R.H00, R.H01, R.S00, R.S01, R.V)
    z = E + 1j * eta
    sigL, sigR = self_energies(z, lead_L, lead_R, eta) if sigma is None else sigma
    Hd, Hu, Sd, Su = dev.blocks()
    Vd, Vu = potential_weights(dev.V, L.V, R.V, dev.pot_mode)
    Ad, Au, Al = assemble(z, Hd, Hu, Sd, Su, Vd, Vu)
    Ad = Ad.copy()
    Ad[0] = Ad[0] - sigL
    Ad[-1] = Ad[-1] - sigR
    return first_block_column(Ad, Au, Al), last_block_column(Ad, Au, Al), broadening(sigL), broadening(sigR)


def contact_blocks(G, gamma):
    """(1/pi) G_{i,X} Gamma_X G_{j,X}^H for j = i (N, m, m) and j = i + 1
    (N-1, m, m), from the block column G_{:,X} of one contact."""
    Gg = G @ gamma                                   # G_{i,X} Gamma_X
    GH = np.swapaxes(G.conj(), -1, -2)               # G_{j,X}^H
    return (Gg @ GH) / np.pi, (Gg[:-1] @ GH[1:]) / np.pi


def density_matrix_blocks(dev, energies, wL, wR, eta):
    """rho_ii (N, m, m) and rho_{i,i+1} (N-1, m, m) over an energy grid
    with per-contact weights (the formula of the module docstring)."""
    energies = np.asarray(energies, dtype=np.float64)
    wL = np.broadcast_to(np.asarray(wL, dtype=np.float64), energies.shape)
    wR = np.broadcast_to(np.asarray(wR, dtype=np.float64), energies.shape)
    N, m = dev.N, dev.m
    rd = np.zeros((N, m, m), dtype=np.complex128)
    ro = np.zeros((max(N - 1, 0), m, m), dtype=np.complex128)
    for E, a, b in zip(energies, wL, wR):
        G0, GN, gL, gR = energy_blocks(dev, float(E), eta)
        for G, g, w in ((G0, gL, a), (GN, gR, b)):
            if w == 0.0:
                continue
            d, o = contact_blocks(G, g)
            rd += w * d
            ro += w * o
    return rd, ro
