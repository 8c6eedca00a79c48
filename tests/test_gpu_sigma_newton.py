"""The Newton step on the lead self-energies (option sigma_newton_tol).

Within about a meV of a band edge of the lead, the doubling decimation
misses the self-energy's fixed point Sigma = A (D0 - Sigma)^-1 B by up to
1e-10 relative (Sec. "Contact self-energies": Sigma is the projection of the
outgoing Bloch modes, which that equation characterises), and the slab
densities inherit the error.  After the doublings every self-energy is
checked against its fixed point and, where the residual exceeds the option
times max|Sigma|, corrected by one Newton step.

Checked against the oracle's self-energy from the complex band structure
(QZ on the lead pencil) on the N = 400, m = 128 lead: uniform energies and
energies within 1 meV of the band edges, among them the worst ones of the
band-edge set.  The corrected GPU self-energy must be within 5e-11 of QZ
(relative to max(1, max|Sigma|)) at every one of them, at least as close as
the oracle's own LAPACK-based decimation wherever that deviates by more
than 5e-11, and switching the step off must leave a larger error at the
worst band-edge energy (so the option reaches the kernel).
"""
import os

import numpy as np
import pytest

from oracle import decimation as odec
from oracle import leads as oleads
from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_SIGMA = 5e-11


def _edges():
    return np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cfg2_band_edge_energies.txt"))


def _rel(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


@pytest.fixture(scope="module")
def m128():
    edges = _edges()
    wl = W.config2(band_edge_energies=edges)
    rng = np.random.default_rng(12)
    n_uni = len(wl.E) - len(edges)
    E = np.concatenate([edges[[254, 150, 250, 11]], edges[rng.choice(len(edges), 8, replace=False)],
                        wl.E[rng.choice(n_uni, 4, replace=False)]])
    dev = wl.device
    ld = (dev.lead_L.H00, dev.lead_L.H01, dev.lead_L.S00, dev.lead_L.S01, dev.lead_L.V)
    qz, dec = [], []
    for e in E:
        z = e + 1j * wl.eta
        qz.append(oleads.self_energies(z, ld, ld, wl.eta))
        dl, dr, _ = odec.decimate(z, ld[:4])
        dec.append((dl, dr))
    return wl, E, qz, dec


def _gpu_errors(wl, E, qz, tol):
    ctx = _lib.context_for(wl.device, 0)
    ctx.set_option("sigma_newton_tol", tol)
    sig, Wf, s, it = ctx.self_energy(E, wl.eta)
    ctx.close()
    assert np.all(np.isfinite(sig))
    return np.array([[_rel(sig[k, side], qz[k][side]) for side in (0, 1)] for k in range(len(E))])


def test_newton_step_reaches_the_band_structure_self_energy(gpu_lib, m128):
    wl, E, qz, dec = m128
    err_on = _gpu_errors(wl, E, qz, 1e-11)
    err_off = _gpu_errors(wl, E, qz, -1.0)
    err_dec = np.array([[_rel(dec[k][side], qz[k][side]) for side in (0, 1)] for k in range(len(E))])
    for k, e in enumerate(E):
        print(f"E={e:+.9f}  GPU+Newton {err_on[k].max():.2e}  GPU doublings only {err_off[k].max():.2e}  "
              f"oracle decimation {err_dec[k].max():.2e}")
    assert err_on.max() <= TOL_SIGMA, err_on.max()
    # as close to QZ as the oracle's LAPACK decimation wherever that is off by more than the bar
    worse = err_dec > TOL_SIGMA
    assert np.all(err_on[worse] <= err_dec[worse])
    assert err_off.max() > err_on.max()


def test_newton_everywhere_keeps_generic_energies(gpu_lib, m128):
    """sigma_newton_tol = 0 corrects every self-energy; at energies where the
    doublings already meet the fixed point the step changes nothing that
    matters (still within the bar of QZ)."""
    wl, E, qz, dec = m128
    err = _gpu_errors(wl, E, qz, 0.0)
    assert err.max() <= TOL_SIGMA, err.max()


def test_newton_option_validation(gpu_lib):
    ctx = _lib.Context(0)
    for bad in (1.0, -2.0, float("nan")):
        with pytest.raises(_lib.QtxError) as ei:
            ctx.set_option("sigma_newton_tol", bad)
        assert ei.value.status == _lib.EINVAL
    for ok in (-1.0, 0.0, 1e-12, 0.5):
        ctx.set_option("sigma_newton_tol", ok)
