"""Energy integrals (density, its potential derivative, current) by the
adaptive driver over the HIP solve, against the oracle's plain composite
Simpson on a uniform grid.  A broadening of 0.05 eV keeps the integrands
smooth on the reference grid; the reference's own error is estimated by
halving its step."""
import numpy as np
import pytest

from oracle import integrals as oint
from oracle.density_matrix import density_matrix_blocks
from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import integrate as I
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu

ETA = 0.05
MUL, MUR, KT = 0.1, -0.1, 0.05


@pytest.fixture(scope="module")
def setup():
    dev = W.small_random_device(51, 10, 8, uniform=False, same_leads=True, pot_mode=W.POT_LINEAR_FE)
    ctx = _lib.context_for(dev, 0)
    return dev, ctx


def _ref(dev, A, B):
    fine = oint.integrals(dev, ETA, A, B, MUL, MUR, KT, 2048)
    coarse = oint.integrals(dev, ETA, A, B, MUL, MUR, KT, 1024)
    return fine, coarse


def test_density_jacobian_current(setup):
    dev, ctx = setup
    solve = I.qtx_solver(ctx, ETA)
    A, B = -7.0, MUL + 20 * KT
    (dens, jac, _), (dens_c, jac_c, _) = _ref(dev, A, B)
    rd = I.integrate(solve, "density", A, B, MUL, MUR, KT, tol=1e-7)
    rj = I.integrate(solve, "jacobian", A, B, MUL, MUR, KT, tol=1e-7)
    assert rd.converged and rj.converged
    for got, ref, refc, name in ((rd.value, dens, dens_c, "density"), (rj.value, jac, jac_c, "jacobian")):
        bar = 10 * np.abs(ref - refc).max() + 1e-6 * max(1.0, np.abs(ref).max())
        err = np.abs(got - ref).max()
        print(f"{name}: max|adaptive - reference| = {err:.2e} (bar {bar:.2e}), {rd.evaluations} energies")
        assert err <= bar
    A2, B2 = MUR - 20 * KT, MUL + 20 * KT
    (_, _, cur), (_, _, cur_c) = _ref(dev, A2, B2)
    rc = I.integrate(solve, "current", A2, B2, MUL, MUR, KT, tol=1e-9)
    bar = 10 * abs(cur - cur_c) + 1e-8
    assert abs(rc.value[0] - cur) <= bar, (rc.value[0], cur, bar)
    # each round is one batched solve of new energies only
    assert rc.rounds <= 40 and len(np.unique(rc.energies)) == rc.evaluations


def test_density_matrix_on_the_adaptive_grid(setup):
    """The density matrix from the energies and quadrature weights of the
    adaptive node-density integration (Sec. "Density": the same points,
    one more pass): the trace of rho_ii equals the integrated density, and
    the blocks equal the oracle's on those energies and weights."""
    dev, ctx = setup
    solve = I.qtx_solver(ctx, ETA)
    A, B = -7.0, MUL + 20 * KT
    r = I.integrate(solve, "density", A, B, MUL, MUR, KT, tol=1e-7)
    rd, ro = I.density_matrix(ctx, r, MUL, MUR, KT, ETA)
    tr = np.real(np.einsum("iaa->i", rd))
    assert np.abs(tr - r.value).max() <= 1e-12 * max(1.0, np.abs(r.value).max())
    E, q = r.energies, r.weights
    ref_d, ref_o = density_matrix_blocks(dev, E, q * I.fermi(E - MUL, KT), q * I.fermi(E - MUR, KT), ETA)
    scale = max(1.0, np.abs(ref_d).max())
    assert np.abs(rd - ref_d).max() <= 1e-9 * scale and np.abs(ro - ref_o).max() <= 1e-9 * scale
