"""Contact self-energies from the complex band structure (oracle, FP64).

Test infrastructure only (see the package docstring).

Conventions.  Slab blocks H00, S00 (on-site) and H01, S01 (coupling from
slab j to slab j+1), z = E + i eta, and for a lead at potential energy V the
shifted z_X = z - V.  With A = zS - H the lead operators are

    D0 = z_X S00 - H00,   U = z_X S01 - H01,   L = z_X S01^H - H01^H,

so L is not U^H when eta > 0.  A Bloch solution obeys c_{j+1} = lambda c_j,
which turns the slab equation into the quadratic eigenvalue problem
[lambda^-1 H_{i,i-1} + H_ii + lambda H_{i,i+1} - z M(lambda)] c = 0
(Sec. "Contact self-energies", eq. complex_bs).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def lead_operators(z, H00, H01, S00, S01, V=0.0):
    """D0, U, L of a lead at potential energy V (conventions above)."""
    zx = z - V
    D0 = zx * S00 - H00
    U = zx * S01 - H01
    L = zx * S01.conj().T - H01.conj().T
    return D0, U, L


def complex_band_modes(z, H00, H01, S00, S01, V=0.0):
    """All 2m Bloch factors lambda and mode vectors c at complex energy z.

    The quadratic problem is linearised with the symmetric scheme of the
    paper (eq. linearized_eigenvalue_symmetric), with d = lambda c:

        [[H00 - zS00, H10 - zS10], [H01 - zS01, 0]] [d; c]
            = lambda [[-(H01 - zS01), 0], [0, H01 - zS01]] [d; c]

    where H10 = H01^H, S10 = S01^H are the couplings to the previous slab.
    Solved with a dense QZ (scipy.linalg.eig on the pencil)."""
    zx = z - V
    m = H00.shape[0]
    Hm = H01.conj().T - zx * S01.conj().T     # H_{i,i-1} - z M_{i,i-1}
    Hp = H01 - zx * S01                       # H_{i,i+1} - z M_{i,i+1}
    H0 = H00 - zx * S00
    Z = np.zeros((m, m), dtype=np.complex128)
    lhs = np.block([[H0, Hm], [Hp, Z]])
    rhs = np.block([[-Hp, Z], [Z, Hp]])
    lam, x = scipy.linalg.eig(lhs, rhs)
    c = x[m:, :]
    return lam, c


def mode_flux(lam, c, U):
    """J = 2 Im(lambda c^H U c) for each column (the numerator of the
    generalised Hellmann-Feynman velocity, eq. hellmann-feynman, at real E)."""
    return 2.0 * np.imag(lam * np.einsum("in,ij,jn->n", c.conj(), U, c))


def mode_mass(lam, c, S00, S01):
    """c^H M(lambda) c with M(lambda) = lambda^-1 S10 + S00 + lambda S01."""
    M = (S00[None] + lam[:, None, None] * S01[None]
         + (1.0 / lam)[:, None, None] * S01.conj().T[None])
    return np.einsum("in,nij,jn->n", c.conj(), M, c)


def classify(lam, c, U, eta, tol=1e-8):
    """Split the 2m modes into right-going (decaying or flowing towards
    +z) and left-going ones.  For eta > 0 the split is |lambda| < 1 alone;
    at eta = 0 modes with ||lambda| - 1| <= tol are travelling and take the
    sign of their flux (Sec. "Contact self-energies", mode split and the
    |lambda| = 1 +- epsilon tolerance).  Returns boolean masks
    (right, left, travelling)."""
    a = np.abs(lam)
    if eta > 0.0:
        right = a < 1.0
        trav = np.zeros_like(right)
    else:
        trav = np.abs(a - 1.0) <= tol
        J = mode_flux(lam, c, U)
        right = (a < 1.0 - tol) | (trav & (J > 0.0))
    left = ~right
    m = c.shape[0]
    if right.sum() != m:
        raise ValueError(f"mode split failed: {right.sum()} right-going of {2*m}")
    return right, left, trav


def bloch_propagators(z, lead, eta, tol=1e-8):
    """F_plus = B+ Lambda+ B+^-1 (maps c_j to c_{j+1} for right-going waves)
    and F_minus_inv = B- Lambda-^-1 B-^-1 (maps c_j to c_{j-1} for
    left-going waves) of one lead."""
    H00, H01, S00, S01, V = lead
    lam, c = complex_band_modes(z, H00, H01, S00, S01, V)
    _, U, _ = lead_operators(z, H00, H01, S00, S01, V)
    right, left, trav = classify(lam, c, U, eta, tol)
    Bp, lp = c[:, right], lam[right]
    Bm, lm = c[:, left], lam[left]
    Fp = np.linalg.solve(Bp.T, (Bp * lp[None, :]).T).T
    Fm_inv = np.linalg.solve(Bm.T, (Bm / lm[None, :]).T).T
    return Fp, Fm_inv


def self_energies(z, lead_L, lead_R, eta, tol=1e-8):
    """Sigma_L, Sigma_R on the first / last device slab.

    Sigma_i = [H'_i - E M'_i] B Lambda B^-1 (Sec. "Contact self-energies"):
    for the drain H' = H_{i,i+1} and the out-flowing modes move towards
    +z, so Sigma_R = (H01 - z S01) F_plus = -U_R F_plus; for the source H' =
    H_{i,i-1} and the out-flowing modes move towards -z, so
    Sigma_L = (H10 - z S10) F_minus^-1 = -L_L F_minus^-1.
    Each lead is a tuple (H00, H01, S00, S01, V)."""
    _, _, L_L = lead_operators(z, *lead_L)
    _, U_R, _ = lead_operators(z, *lead_R)
    _, FmL_inv = bloch_propagators(z, lead_L, eta, tol)
    FpR, _ = bloch_propagators(z, lead_R, eta, tol)
    sigL = -L_L @ FmL_inv
    sigR = -U_R @ FpR
    return sigL, sigR


def broadening(sigma):
    """Gamma = i (Sigma - Sigma^H)."""
    return 1j * (sigma - sigma.conj().T)


def open_channels(E, lead, tol=1e-8):
    """Number of travelling right-going modes of a lead at real energy E."""
    H00, H01, S00, S01, V = lead
    lam, c = complex_band_modes(E + 0j, H00, H01, S00, S01, V)
    _, U, _ = lead_operators(E + 0j, H00, H01, S00, S01, V)
    right, _, trav = classify(lam, c, U, 0.0, tol)
    return int(np.sum(right & trav))
