"""The paper's own mode-space QTBM at eta = 0 (oracle cross-check, FP64).

Test infrastructure only (see the package docstring).

Steps, in the paper's order (Sec. "Contact self-energies", "Extended
states", "Density", "Transmission and Ballistic Current"):

1. complex band structure of each contact at real E (oracle.leads);
2. travelling modes are those with |lambda| = 1 within a tolerance, their
   direction is the sign of the Hellmann-Feynman velocity
   v = [c^H dH/dk c - E c^H dM/dk c] / (c^H M(lambda) c)
   (eq. hellmann-feynman; its numerator is the flux 2 Im(lambda c^H U c));
3. travelling modes are normalised to c^H M(lambda) c = L_z / (2 pi) with
   L_z = 1 (eq. normalization);
4. each incoming mode gamma of the source is injected with the right-hand
   side B_gamma = [(H' - E M') lambda_gamma - Sigma] c_gamma on the first
   slab (H' = H_{i,i-1}), i.e. (-L lambda^-1 - Sigma_L) c_gamma in the
   A = zS - H convention, and [EM - H - Sigma] c = B is solved
   (eq. qtbm_system);
5. T_gamma = sum_mu |[B_d^-1 c_d]_mu|^2 v_mu / v_gamma over the drain's
   out-flowing travelling modes (eq. transmission); the reflection uses the
   source's out-flowing modes after removing the injected wave; T + R = 1;
6. node density n_i = sum_gamma g_gamma sum_{j in slab i} |c_{gamma,j}|^2
   with g_gamma = 2/|v_gamma| (spin 2), and the nearest-neighbour blocks of
   the density matrix per contact, sum_gamma g_gamma c_{gamma,i} c_{gamma,j}^H
   for j = i, i + 1 (eq. density_matrices at one energy, unit weight and
   occupation; the paper's index order is the transpose).
"""
from __future__ import annotations

import numpy as np

from .leads import (lead_operators, complex_band_modes, classify, mode_flux,
                    mode_mass, self_energies, broadening)
from .device import potential_weights, assemble, first_block_column, last_block_column


def _modes(E, lead, tol):
    H00, H01, S00, S01, V = lead
    z = E + 0j
    lam, c = complex_band_modes(z, H00, H01, S00, S01, V)
    _, U, _ = lead_operators(z, H00, H01, S00, S01, V)
    right, left, trav = classify(lam, c, U, 0.0, tol)
    J = mode_flux(lam, c, U)
    mass = np.real(mode_mass(lam, c, S00, S01))
    c = c.copy()
    v = np.zeros(lam.shape[0])
    for n in np.nonzero(trav)[0]:
        c[:, n] *= np.sqrt((1.0 / (2.0 * np.pi)) / mass[n])
        v[n] = J[n] / mass[n]
    return dict(lam=lam, c=c, right=right, left=left, trav=trav, v=v)


def qtbm_energy(dev, E, tol=1e-8):
    """Mode-space transport at real E: dict with T_LR, R_LR, T_RL, R_RL
    (summed over injected modes), per-mode arrays, the node densities
    n^L, n^R (N,), and the open-channel counts."""
    L, R = dev.lead_L, dev.lead_R
    lead_L = (L.H00, L.H01, L.S00, L.S01, L.V)
    lead_R = (R.H00, R.H01, R.S00, R.S01, R.V)
    z = E + 0j
    sigL, sigR = self_energies(z, lead_L, lead_R, 0.0, tol)
    Hd, Hu, Sd, Su = dev.blocks()
    Vd, Vu = potential_weights(dev.V, L.V, R.V, dev.pot_mode)
    Ad, Au, Al = assemble(z, Hd, Hu, Sd, Su, Vd, Vu)
    Ad = Ad.copy()
    Ad[0] -= sigL
    Ad[-1] -= sigR
    G0 = first_block_column(Ad, Au, Al)
    GN = last_block_column(Ad, Au, Al)
    mL = _modes(E, lead_L, tol)
    mR = _modes(E, lead_R, tol)
    _, _, L_L = lead_operators(z, *lead_L)
    _, U_R, _ = lead_operators(z, *lead_R)

    BpR = mR["c"][:, mR["right"]]            # drain out-flowing Bloch matrix
    propR = mR["trav"][mR["right"]]
    vR_out = mR["v"][mR["right"]]
    BmL = mL["c"][:, mL["left"]]             # source out-flowing Bloch matrix
    propL = mL["trav"][mL["left"]]
    vL_out = mL["v"][mL["left"]]

    N = dev.N
    m = dev.m
    out = dict(T_LR=[], R_LR=[], T_RL=[], R_RL=[], v_inj_L=[], v_inj_R=[],
               nL=np.zeros(N), nR=np.zeros(N), B_L=[], B_R=[],
               rhoL_d=np.zeros((N, m, m), complex), rhoL_o=np.zeros((N - 1, m, m), complex),
               rhoR_d=np.zeros((N, m, m), complex), rhoR_o=np.zeros((N - 1, m, m), complex))

    def add_blocks(key, g, c):
        out[key + "_d"] += g * np.einsum("ia,ib->iab", c, c.conj())
        out[key + "_o"] += g * np.einsum("ia,ib->iab", c[:-1], c[1:].conj())
    # injection from the source: incoming = right-going travelling modes
    for g in np.nonzero(mL["right"] & mL["trav"])[0]:
        cg, lg, vg = mL["c"][:, g], mL["lam"][g], mL["v"][g]
        B = (-L_L / lg - sigL) @ cg
        c = G0 @ B                              # (N, m): solution on all slabs
        a = np.linalg.solve(BpR, c[-1])
        T = np.sum(np.abs(a[propR]) ** 2 * vR_out[propR]) / vg
        r = np.linalg.solve(BmL, c[0] - cg)
        Rf = np.sum(np.abs(r[propL]) ** 2 * np.abs(vL_out[propL])) / vg
        out["T_LR"].append(T)
        out["R_LR"].append(Rf)
        out["v_inj_L"].append(vg)
        out["B_L"].append(B)
        out["nL"] += (2.0 / abs(vg)) * np.sum(np.abs(c) ** 2, axis=1)
        add_blocks("rhoL", 2.0 / abs(vg), c)
    # injection from the drain: incoming = left-going travelling modes
    for g in np.nonzero(mR["left"] & mR["trav"])[0]:
        cg, lg, vg = mR["c"][:, g], mR["lam"][g], mR["v"][g]
        B = (-U_R * lg - sigR) @ cg
        c = GN @ B
        a = np.linalg.solve(BmL, c[0])
        T = np.sum(np.abs(a[propL]) ** 2 * np.abs(vL_out[propL])) / abs(vg)
        r = np.linalg.solve(BpR, c[-1] - cg)
        Rf = np.sum(np.abs(r[propR]) ** 2 * vR_out[propR]) / abs(vg)
        out["T_RL"].append(T)
        out["R_RL"].append(Rf)
        out["v_inj_R"].append(vg)
        out["B_R"].append(B)
        out["nR"] += (2.0 / abs(vg)) * np.sum(np.abs(c) ** 2, axis=1)
        add_blocks("rhoR", 2.0 / abs(vg), c)
    out["n_open_L"] = len(out["T_LR"])
    out["n_open_R"] = len(out["T_RL"])
    out["gamma_L"] = broadening(sigL)
    out["gamma_R"] = broadening(sigR)
    out["G0"], out["GN"] = G0, GN
    return out
