"""The oracle's own error bar at the full workload sizes.

No closed form exists for the N = 200, m = 64 and N = 400, m = 128
workloads, so the oracle checks itself there: its right-connected block
elimination and its two-pass elimination (the opposite order for the first
block column) must agree on sampled energies, and their spread is the
oracle's error bar at those sizes.  Measured on these samples: |dT| up to
3.9e-12; slab densities up to 7.6e-9 (N = 200) and 3.9e-8 (N = 400)
absolute where single-energy densities reach 300-450 states / eV / slab,
i.e. up to 1e-10 relative.  The bars asserted here are the GPU parity bars
(|dT| <= 1e-10, |dn| <= 1e-9 relative); the absolute spread is printed.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1903_00548_amd import workloads as W


def _spread(dev, energies, eta):
    dT, rel, ab = 0.0, 0.0, 0.0
    for e in energies:
        a = oracle.solve_energy(dev, float(e), eta, method="right")
        b = oracle.solve_energy(dev, float(e), eta, method="two_pass")
        scale = max(1.0, np.abs(a[1]).max(), np.abs(a[2]).max())
        d = max(np.abs(a[1] - b[1]).max(), np.abs(a[2] - b[2]).max())
        dT, rel, ab = max(dT, abs(a[0] - b[0])), max(rel, d / scale), max(ab, d)
    return dT, rel, ab


def test_elimination_orders_agree_headline_grid():
    wl = W.config1()
    rng = np.random.default_rng(2024)
    idx = np.concatenate([[768], rng.choice(len(wl.E), 7, replace=False)])
    dT, rel, ab = _spread(wl.device, wl.E[idx], wl.eta)
    print(f"N=200 m=64, 8 energies: max|dT| {dT:.2e}, max rel|dn| {rel:.2e}, max abs|dn| {ab:.2e}")
    assert dT <= 1e-10 and rel <= 1e-9


def test_elimination_orders_agree_large_grid_band_edge():
    edges = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cfg2_band_edge_energies.txt"))
    wl = W.config2(band_edge_energies=edges)
    E = np.array([wl.E[7], edges[150]])          # a uniform energy and one within 1 meV of a band edge
    dT, rel, ab = _spread(wl.device, E, wl.eta)
    print(f"N=400 m=128, 2 energies: max|dT| {dT:.2e}, max rel|dn| {rel:.2e}, max abs|dn| {ab:.2e}")
    assert dT <= 1e-10 and rel <= 1e-9
