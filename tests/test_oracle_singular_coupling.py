"""Leads whose slab coupling U = z S01 - H01 is singular (fewer coupling
directions than orbitals per slab).

* The paper's symmetric linearisation (eq. linearized_eigenvalue_symmetric)
  is then a singular pencil: its determinant carries det U as a factor, so
  it vanishes at every lambda and the pencil's eigenvalues are not
  defined.  This is why the GPU's direct method solves the quadratic in a
  shifted variable instead (checked in tests/test_gpu_modes.py).
* The oracle's decimation needs no inverse of U; it is pinned here to the
  closed form of a chain with one side orbital per slab (coupling of rank
  one, tests/side_chain.py).
"""
import numpy as np
import pytest

from oracle import decimation as odec
from oracle import leads as oleads
from paper_1903_00548_amd import workloads as W

import side_chain


def _pencil(z, lead):
    H00, H01, S00, S01, Vl = lead
    zx = z - Vl
    m = H00.shape[0]
    Hm = H01.conj().T - zx * S01.conj().T
    Hp = H01 - zx * S01
    Z = np.zeros((m, m), complex)
    return np.block([[H00 - zx * S00, Hm], [Hp, Z]]), np.block([[-Hp, Z], [Z, Hp]])


@pytest.mark.parametrize("rank", [2, 4])
def test_paper_pencil_is_singular_when_the_coupling_is(rank):
    rng = np.random.default_rng(40 + rank)
    ld = W.low_rank_coupling_lead(rng, 6, rank)
    lead = (ld.H00, ld.H01, ld.S00, ld.S01, ld.V)
    full = W.random_lead(np.random.default_rng(7), 6)
    for lam in (0.3, 1.7 + 0.2j, -2.0 - 0.5j):
        A, B = _pencil(0.4 + 0j, lead)
        sv = np.linalg.svd(A - lam * B, compute_uv=False)
        assert sv[-1] <= 1e-13 * sv[0], (rank, lam, sv[-1] / sv[0])
        A, B = _pencil(0.4 + 0j, (full.H00, full.H01, full.S00, full.S01, 0.0))
        sv = np.linalg.svd(A - lam * B, compute_uv=False)
        assert sv[-1] >= 1e-6 * sv[0]
    U = 0.4 * ld.S01 - ld.H01
    assert np.linalg.matrix_rank(U) == rank


@pytest.mark.parametrize("E", [-2.6, -1.2, 0.4, 1.5, 2.5])
def test_decimation_matches_side_chain_closed_form(E):
    for eta in (1e-6, 1e-9):
        z = E + 1j * eta
        sL, sR, it = odec.decimate(z, side_chain.lead())
        ref = side_chain.sigma(z)
        scale = np.abs(ref).max()
        assert np.abs(sR - ref).max() <= 1e-10 * scale, (E, eta)
        assert np.abs(sL - ref).max() <= 1e-10 * scale, (E, eta)
        assert -ref[0, 0].imag >= 0.0                   # retarded: Gamma >= 0


def test_closed_form_catches_a_dropped_side_orbital():
    """The pin is sharp: without the side orbital the chain's Sigma differs
    by far more than the bar inside the band."""
    z = 0.4 + 1e-9j
    H00, H01, S00, S01, _ = side_chain.lead()
    bare = (np.diag([side_chain.EA, side_chain.EB]).astype(complex), H01, S00, S01, 0.0)
    sL, sR, it = odec.decimate(z, bare)
    assert np.abs(sR - side_chain.sigma(z)).max() > 1e-3
