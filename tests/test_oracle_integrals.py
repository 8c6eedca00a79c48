"""Pins of the oracle's energy integrals (oracle.integrals.integrals)
against closed forms, and planted mistakes that the pins must catch.

The pinned system is a perfect one-band chain (m = 1, on-site 0, hopping
-t, orthogonal basis) at eta = 0, a device that copies its leads.  Inside
the band |E| < 2t:
  * T(E) = 1 exactly (one open channel, no scattering), so the current
    integral is J = int_A^B [f_L - f_R] dE, and with the antiderivative
    F_mu(E) = E - kT ln(1 + exp((E - mu)/kT)) of the Fermi function this
    is F_muL(B) - F_muL(A) - F_muR(B) + F_muR(A) in closed form;
  * the slab density of the states injected by either contact is the
    chain's density of right- (or left-) moving states, with spin 2,
    h(E) = 1 / (pi sqrt(4t^2 - E^2)) per slab, whose antiderivative is
    H(E) = arcsin(E/2t) / pi.  With f the Fermi function, the Sommerfeld
    expansion gives int_A^B f(E - mu) h(E) dE = H(mu) - H(A)
    + (pi^2/6) kT^2 h'(mu) + O(kT^4) when A lies many kT below mu and B
    many kT above it, and for the Jacobian int (-f') h dE = h(mu)
    + (pi^2/6) kT^2 h''(mu) + O(kT^4).
With mu_L != mu_R the current changes sign when the contacts' occupations
are exchanged, so an f_L / f_R swap fails the current pin; a dropped
contact term halves the density; a sign slip in -df/dE flips the Jacobian.
"""
import numpy as np
import pytest

from oracle import integrals as oint
from oracle.device import POT_DIAG
from paper_1903_00548_amd import workloads as W

T_HOP = 1.0
A, B = -1.5, 1.5
MU_L, MU_R, KT = 0.3, -0.2, 0.01
NINT = 2400


def _chain(N=4):
    lead = W.Lead(H00=np.zeros((1, 1), complex), H01=-T_HOP * np.ones((1, 1), complex),
                  S00=np.eye(1, dtype=complex), S01=np.zeros((1, 1), complex))
    return W.Device(N=N, m=1, lead_L=lead, lead_R=lead, V=np.zeros(N), pot_mode=POT_DIAG)


def _h(E):
    return 1.0 / (np.pi * np.sqrt(4 * T_HOP ** 2 - E ** 2))


def _h1(E):
    return E / (np.pi * (4 * T_HOP ** 2 - E ** 2) ** 1.5)


def _h2(E):
    s = 4 * T_HOP ** 2 - E ** 2
    return (s + 3 * E ** 2) / (np.pi * s ** 2.5)


def _F(E, mu):
    return E - KT * np.logaddexp(0.0, (E - mu) / KT)


def expected():
    H = lambda E: np.arcsin(E / (2 * T_HOP)) / np.pi
    dens = sum(H(mu) - H(A) + np.pi ** 2 / 6 * KT ** 2 * _h1(mu) for mu in (MU_L, MU_R))
    jac = sum(_h(mu) + np.pi ** 2 / 6 * KT ** 2 * _h2(mu) for mu in (MU_L, MU_R))
    cur = _F(B, MU_L) - _F(A, MU_L) - _F(B, MU_R) + _F(A, MU_R)
    return dens, jac, cur


def pins_ok():
    dev = _chain()
    dens, jac, cur = oint.integrals(dev, 0.0, A, B, MU_L, MU_R, KT, NINT)
    d0, j0, c0 = expected()
    return (abs(cur - c0) <= 1e-9 and np.abs(dens - d0).max() <= 1e-8
            and np.abs(jac - j0).max() <= 1e-6 * j0)


def test_closed_forms_hold():
    dev = _chain()
    dens, jac, cur = oint.integrals(dev, 0.0, A, B, MU_L, MU_R, KT, NINT)
    d0, j0, c0 = expected()
    assert abs(cur - c0) <= 1e-9, (cur, c0)
    assert abs(c0 - (MU_L - MU_R)) < 1e-12          # the window holds both Fermi steps
    assert np.abs(dens - d0).max() <= 1e-8, (dens, d0)
    assert np.abs(jac - j0).max() <= 1e-6 * j0, (jac, j0)
    # every slab of a perfect chain carries the same density
    assert np.ptp(dens) < 1e-12 and np.ptp(jac) < 1e-10


def _swapped_occupations(dev, eta, A_, B_, muL, muR, kT, n):
    E = np.linspace(A_, B_, n + 1)
    T, L = oint.solve_device(dev, E, eta)
    w = oint.simpson_weights(A_, B_, n)
    fL, fR = oint.fermi(E, muR, kT), oint.fermi(E, muL, kT)
    gL, gR = oint.minus_dfermi(E, muR, kT), oint.minus_dfermi(E, muL, kT)
    dens = (w * fL) @ L[:, 0, :] + (w * fR) @ L[:, 1, :]
    jac = (w * gL) @ L[:, 0, :] + (w * gR) @ L[:, 1, :]
    return dens, jac, float(np.sum(w * T * (fL - fR)))


def _right_contact_dropped(dev, eta, A_, B_, muL, muR, kT, n):
    E = np.linspace(A_, B_, n + 1)
    T, L = oint.solve_device(dev, E, eta)
    w = oint.simpson_weights(A_, B_, n)
    fL, fR = oint.fermi(E, muL, kT), oint.fermi(E, muR, kT)
    gL = oint.minus_dfermi(E, muL, kT)
    return (w * fL) @ L[:, 0, :], (w * gL) @ L[:, 0, :], float(np.sum(w * T * (fL - fR)))


def _jacobian_sign(dev, eta, A_, B_, muL, muR, kT, n):
    d, j, c = _orig(dev, eta, A_, B_, muL, muR, kT, n)
    return d, -j, c


def _trapezoid_weights(A_, B_, n):
    w = np.full(n + 1, (B_ - A_) / n)
    w[0] = w[-1] = 0.5 * (B_ - A_) / n
    return w * 1.001


_orig = oint.integrals

MUTATIONS = {
    "contact occupations swapped": [(oint, "integrals", _swapped_occupations)],
    "right-injected density dropped": [(oint, "integrals", _right_contact_dropped)],
    "jacobian sign": [(oint, "integrals", _jacobian_sign)],
    "quadrature weights off": [(oint, "simpson_weights", _trapezoid_weights)],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    for mod, attr, fn in MUTATIONS[name]:
        monkeypatch.setattr(mod, attr, fn)
    assert not pins_ok(), f"mutation '{name}' went undetected"
