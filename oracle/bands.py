"""Lead band structure from the Bloch-theorem eigenproblem (oracle, FP64).

Test infrastructure only.

With c_{j+1} = e^{ik} c_j the slab equations reduce to the generalised
Hermitian eigenproblem H(k) c = E S(k) c with
H(k) = H00 + H01 e^{ik} + H01^H e^{-ik} and S(k) likewise (Sec. "Results:
Graphene Nanoribbon", band-structure reconstruction).  Used to count open
channels independently of the complex band structure and to locate band
extrema (energies of vanishing group velocity).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.optimize


def bloch_matrices(k, H00, H01, S00, S01):
    e = np.exp(1j * k)
    Hk = H00 + H01 * e + H01.conj().T / e
    Sk = S00 + S01 * e + S01.conj().T / e
    return 0.5 * (Hk + Hk.conj().T), 0.5 * (Sk + Sk.conj().T)


def bands(k_grid, H00, H01, S00, S01, V=0.0):
    """Sorted band energies E_n(k) + V, shape (len(k_grid), m)."""
    out = np.empty((len(k_grid), H00.shape[0]))
    for a, k in enumerate(k_grid):
        Hk, Sk = bloch_matrices(k, H00, H01, S00, S01)
        out[a] = scipy.linalg.eigh(Hk, Sk, eigvals_only=True)
    return out + V


def open_channels_scan(E, H00, H01, S00, S01, V=0.0, nk=4096):
    """Number of right-going travelling modes at E = number of up-crossings
    of E by the bands over one period.  Counted as half the total number
    of changes of #{n : E_n(k) < E} around the periodic k grid."""
    k = -np.pi + 2.0 * np.pi * np.arange(nk) / nk
    eb = bands(k, H00, H01, S00, S01, V)
    below = np.sum(eb < E, axis=1)
    changes = np.abs(np.diff(np.concatenate([below, below[:1]]))).sum()
    return int(changes // 2)


def _band_slope(k, n, H00, H01, S00, S01):
    """dE_n/dk by the Hellmann-Feynman form c^H (H'(k) - E S'(k)) c / c^H S c."""
    Hk, Sk = bloch_matrices(k, H00, H01, S00, S01)
    w, v = scipy.linalg.eigh(Hk, Sk)
    e = np.exp(1j * k)
    dH = 1j * (H01 * e - H01.conj().T / e)
    dS = 1j * (S01 * e - S01.conj().T / e)
    c = v[:, n]
    num = c.conj() @ (dH - w[n] * dS) @ c
    den = c.conj() @ Sk @ c
    return float(np.real(num / den))


def band_extrema(H00, H01, S00, S01, V=0.0, nk=4096, window=(-1.5, 1.5)):
    """Energies of the band extrema inside `window`: local extrema of each
    sorted band on a k grid, refined with Brent's method on the
    Hellmann-Feynman slope to 1e-12 in k."""
    k = -np.pi + 2.0 * np.pi * np.arange(nk) / nk
    eb = bands(k, H00, H01, S00, S01, 0.0)
    dk = 2.0 * np.pi / nk
    out = []
    m = H00.shape[0]
    for n in range(m):
        e = eb[:, n]
        if e.max() + V < window[0] - 0.01 or e.min() + V > window[1] + 0.01:
            continue
        prev = np.roll(e, 1)
        nxt = np.roll(e, -1)
        idx = np.nonzero(((e >= prev) & (e >= nxt)) | ((e <= prev) & (e <= nxt)))[0]
        for i in idx:
            a, b = k[i] - dk, k[i] + dk
            fa = _band_slope(a, n, H00, H01, S00, S01)
            fb = _band_slope(b, n, H00, H01, S00, S01)
            if fa * fb < 0.0:
                kk = scipy.optimize.brentq(_band_slope, a, b,
                                           args=(n, H00, H01, S00, S01), xtol=1e-12)
            else:
                kk = k[i]
            Hk, Sk = bloch_matrices(kk, H00, H01, S00, S01)
            ee = scipy.linalg.eigh(Hk, Sk, eigvals_only=True)[n] + V
            if window[0] <= ee <= window[1]:
                out.append(ee)
    return np.unique(np.round(np.array(out), 12))
