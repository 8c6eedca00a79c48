"""The slab charge against the oracle at 1e-8 absolute.

charge_i = sum_k w_k [f_L(E_k) n^L_i(E_k) + f_R(E_k) n^R_i(E_k)]: the
energy-integrated, Fermi-weighted node density (Sec. "Density", eq.
density_3d at the nodes), formed by the library's qtx_charge from the
densities of a GPU solve and by the test from the oracle's densities with
the oracle's Fermi function.  FP64 and mixed precision, on a dense grid of
the tiny workload with Simpson weights, and on the N = 200, m = 64 grid
(sampled energies with the grid spacing as weight, and every energy for
mixed against FP64, the FP64 path being held to the oracle by the parity
tests)."""
import numpy as np
import pytest

import oracle
from oracle import integrals as oint
from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_Q = 1e-8
MU_L, MU_R, KT = 0.2, -0.1, 0.025


def _oracle_charge(ldos, w, E):
    fL, fR = oint.fermi(E, MU_L, KT), oint.fermi(E, MU_R, KT)
    return (w * fL) @ ldos[:, 0, :] + (w * fR) @ ldos[:, 1, :]


@pytest.mark.parametrize("prec", [_lib.FP64, _lib.MIXED], ids=["fp64", "mixed"])
def test_charge_dense_grid_tiny(gpu_lib, prec):
    wl = W.config0()
    E = np.linspace(-3.0, 3.0, 401)
    w = oint.simpson_weights(-3.0, 3.0, 400)
    ctx = _lib.context_for(wl.device, 0)
    T, L, info, st = ctx.solve(E, wl.eta, prec)
    q = _lib.charge(L, w, E, MU_L, MU_R, KT)
    _, Lref = oracle.solve_device(wl.device, E, wl.eta)
    qref = _oracle_charge(Lref, w, E)
    d = np.abs(q - qref).max()
    print(f"tiny grid charge: max|dq| = {d:.3e} (max q {np.abs(qref).max():.3f})")
    assert d <= TOL_Q, d


def test_charge_headline_grid(gpu_lib):
    wl = W.config1()
    dev = wl.device
    ctx = _lib.context_for(dev, 0)
    T64, L64, _, _ = ctx.solve(wl.E, wl.eta, _lib.FP64)
    Tm, Lm, _, _ = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    dE = wl.E[1] - wl.E[0]
    rng = np.random.default_rng(99)
    idx = np.sort(rng.choice(len(wl.E), 24, replace=False))
    _, Lref = oracle.solve_device(dev, wl.E[idx], wl.eta)
    w = np.full(len(idx), dE)
    qref = _oracle_charge(Lref, w, wl.E[idx])
    for name, L in (("fp64", L64), ("mixed", Lm)):
        q = _lib.charge(L[idx], w, wl.E[idx], MU_L, MU_R, KT)
        d = np.abs(q - qref).max()
        print(f"N=200 m=64 {name}, 24 sampled energies: max|dq| = {d:.3e} (max q {np.abs(qref).max():.3f})")
        assert d <= TOL_Q, (name, d)
    # every energy of the grid: mixed against FP64
    wall = oint.simpson_weights(wl.E[0], wl.E[-1], len(wl.E) - 1) if len(wl.E) % 2 else np.full(len(wl.E), dE)
    q64 = _lib.charge(L64, wall, wl.E, MU_L, MU_R, KT)
    qm = _lib.charge(Lm, wall, wl.E, MU_L, MU_R, KT)
    d = np.abs(qm - q64).max()
    print(f"N=200 m=64 mixed vs fp64, all 2048 energies: max|dq| = {d:.3e} (max q {np.abs(q64).max():.3f})")
    assert d <= TOL_Q, d
