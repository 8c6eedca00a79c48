"""Independent lead self-energy references (oracle pins, FP64).

Test infrastructure only.  Two routes to the same Sigma as oracle.leads,
written separately so that each can pin the other:

* `decimate`: the doubling (cyclic-reduction) elimination of every other
  slab of the semi-infinite lead, iterated until the couplings vanish;
* `brute_force_lead`: the plain linear recursion g <- (D0 - U g L)^-1, i.e.
  a finite lead grown one slab at a time; only usable at a large
  broadening where it converges within a few thousand slabs.

Both use the conventions of oracle.leads (A = zS - H; U couples slab j to
j+1 and L couples j+1 back to j).  Sigma_R = U g_R L with g_R = (D0 - U g_R
L)^-1, and Sigma_L = L g_L U with g_L = (D0 - L g_L U)^-1.
"""
from __future__ import annotations

import numpy as np

from .leads import lead_operators


def decimate(z, lead, tol=1e-14, max_iter=200):
    """Returns (Sigma_L-type, Sigma_R-type, iterations) for ONE lead: the
    self-energy this lead would give if attached on the left, and on the
    right.  Eliminating the odd slabs of a chain with on-site e and
    couplings a (forward) and b (backward) gives
    e' = e - a e^-1 b - b e^-1 a, a' = -a e^-1 a, b' = -b e^-1 b; the
    surface of a right lead only loses a e^-1 b and the surface of a left
    lead only b e^-1 a."""
    D0, U, L = lead_operators(z, *lead)
    e = D0.copy()
    esR = D0.copy()
    esL = D0.copy()
    a = U.copy()
    b = L.copy()
    scale = np.linalg.norm(D0, 1)
    for it in range(1, max_iter + 1):
        ga = np.linalg.solve(e, a)
        gb = np.linalg.solve(e, b)
        agb = a @ gb
        bga = b @ ga
        esR = esR - agb
        esL = esL - bga
        e = e - agb - bga
        a = -a @ ga
        b = -b @ gb
        if np.linalg.norm(a, 1) + np.linalg.norm(b, 1) < tol * scale:
            break
    return D0 - esL, D0 - esR, it


def brute_force_lead(z, lead, n_slabs=4000):
    """Sigma_L-type and Sigma_R-type by growing a finite lead slab by slab."""
    D0, U, L = lead_operators(z, *lead)
    gR = np.linalg.inv(D0)
    gL = np.linalg.inv(D0)
    for _ in range(n_slabs):
        gR = np.linalg.inv(D0 - U @ gR @ L)
        gL = np.linalg.inv(D0 - L @ gL @ U)
    return L @ gL @ U, U @ gR @ L
