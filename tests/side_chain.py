"""A chain with one side orbital per slab: the chain orbital a (level e_a)
couples to its neighbours by t, the side orbital b (level e_b) only to a in
its own slab (by v), so the slab coupling H01 has rank one.  Eliminating b
gives the chain the on-site level e_eff(z) = e_a + v^2 / (z - e_b); the
surface Green's function of a semi-infinite chain with hopping t is the
root g of t^2 g^2 - (z - e_eff) g + 1 = 0 with |t g| <= 1 (in the band: the
one with Im g < 0), and Sigma = t^2 g on the chain orbital of the contact
slab, zero elsewhere, for either lead.  Test data only."""
import numpy as np

EA, EB, V, T = 0.1, -0.3, 0.25, -1.0


def lead():
    """(H00, H01, S00, S01, V_lead)."""
    H00 = np.array([[EA, V], [V, EB]], complex)
    H01 = np.array([[T, 0.0], [0.0, 0.0]], complex)
    return (H00, H01, np.eye(2, dtype=complex), np.zeros((2, 2), complex), 0.0)


def sigma(z):
    d = z - (EA + V * V / (z - EB))
    r = np.sqrt(d * d - 4 * T * T + 0j)
    g1, g2 = (d - r) / (2 * T * T), (d + r) / (2 * T * T)
    g = g1 if abs(T * g1) < abs(T * g2) else g2
    if abs(abs(T * g1) - abs(T * g2)) < 1e-9:      # in the band: the retarded root
        g = g1 if g1.imag < 0 else g2
    s = np.zeros((2, 2), complex)
    s[0, 0] = T * T * g
    return s


def open_channels(E):
    """1 inside the chain's band |E - e_eff(E)| < 2|t|, else 0."""
    return int(abs(E - (EA + V * V / (E - EB))) < 2 * abs(T))
