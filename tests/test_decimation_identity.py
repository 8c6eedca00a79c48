"""The decimation kernel stores only e and the right surface block e_R and
forms Sigma_L = e_R - e (Sec. "Contact self-energies": the surface blocks of
the semi-infinite leads).  This rests on an identity of the doubling: each
step subtracts a g b from e and from e_R, and b g a from e and from the left
surface block e_L.  So e_L = e + D0 - e_R holds at every step.  Checked here
on a plain FP64 doubling that tracks all three blocks, and at convergence
against the oracle's complex-band-structure self-energies."""
import numpy as np
import pytest

from oracle import leads
from paper_1903_00548_amd import workloads as W


@pytest.mark.parametrize("m,E,eta", [(4, 0.3, 1e-3), (8, -1.1, 1e-4), (6, 2.2, 1e-2)])
def test_left_surface_from_e_and_right_surface(m, E, eta):
    lead = W.random_lead(np.random.default_rng(100 + m), m)
    z = E + 1j * eta
    D0, U, L = leads.lead_operators(z, lead.H00, lead.H01, lead.S00, lead.S01)
    e, eL, eR, a, b = D0.copy(), D0.copy(), D0.copy(), U.copy(), L.copy()
    scale = np.abs(D0).max()
    for _ in range(200):
        g = np.linalg.inv(e)
        agb, bga = a @ g @ b, b @ g @ a
        e, eR, eL = e - agb - bga, eR - agb, eL - bga
        a, b = -a @ g @ a, -b @ g @ b
        assert np.abs(eL - (e + D0 - eR)).max() <= 1e-12 * scale
        if np.abs(a).max() + np.abs(b).max() < 1e-15 * scale:
            break
    sL_ref, sR_ref = leads.self_energies(z, (lead.H00, lead.H01, lead.S00, lead.S01, 0.0),
                                         (lead.H00, lead.H01, lead.S00, lead.S01, 0.0), eta)
    ref = max(1.0, np.abs(sL_ref).max())
    assert np.abs((eR - e) - sL_ref).max() <= 1e-9 * ref
    assert np.abs((D0 - eL) - sL_ref).max() <= 1e-9 * ref
    assert np.abs((D0 - eR) - sR_ref).max() <= 1e-9 * max(1.0, np.abs(sR_ref).max())
