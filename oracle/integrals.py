"""Energy integrals of the transport quantities (oracle, FP64).

Test infrastructure only (see the package docstring).

Written from their definitions: the node density of injected states
weighted by each contact's Fermi function (Sec. "Density", eq.
density_3d), its derivative with respect to the electrochemical potential
(eq. density_jacobian, taken as d n / d mu, i.e. with -df/dE), and the
ballistic current integral J = int T(E) [f_L - f_R] dE (eq. current), by
the plain composite Simpson rule on a uniform grid of 2K + 1 energies.
"""
from __future__ import annotations

import numpy as np

from .observables import solve_device


def fermi(E, mu, kT):
    x = np.clip((np.asarray(E, dtype=float) - mu) / kT, -700.0, 700.0)
    return 1.0 / (1.0 + np.exp(x))


def minus_dfermi(E, mu, kT):
    # -df/dE = e^x / (1 + e^x)^2 / kT, symmetric in x; written with
    # e^{-|x|} so that neither tail cancels
    t = np.exp(-np.abs(np.clip((np.asarray(E, dtype=float) - mu) / kT, -700.0, 700.0)))
    return t / (1.0 + t) ** 2 / kT


def simpson_weights(A, B, n_intervals):
    """Composite Simpson weights for n_intervals (even) equal intervals."""
    if n_intervals % 2:
        raise ValueError("Simpson needs an even number of intervals")
    h = (B - A) / n_intervals
    w = np.full(n_intervals + 1, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    return w * h / 3.0


def integrals(dev, eta, A, B, muL, muR, kT, n_intervals):
    """density (N,), jacobian (N,), current J (eV) on a uniform grid."""
    E = np.linspace(A, B, n_intervals + 1)
    T, L = solve_device(dev, E, eta)
    w = simpson_weights(A, B, n_intervals)
    fL, fR = fermi(E, muL, kT), fermi(E, muR, kT)
    gL, gR = minus_dfermi(E, muL, kT), minus_dfermi(E, muR, kT)
    dens = (w * fL) @ L[:, 0, :] + (w * fR) @ L[:, 1, :]
    jac = (w * gL) @ L[:, 0, :] + (w * gR) @ L[:, 1, :]
    cur = float(np.sum(w * T * (fL - fR)))
    return dens, jac, cur
