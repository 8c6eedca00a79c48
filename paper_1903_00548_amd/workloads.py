"""Seeded synthetic inputs for the open-boundary transport solve.

This module only draws random numbers and arranges them into the block
matrices, potentials and energy grids that both the HIP path and the CPU
oracle consume.  It holds none of the method's arithmetic (no self-energies,
no solves, no observables).

The paper's own workload is a graphene-nanoribbon FET whose Bloch-wave
matrices come from empirical pseudopotentials (Sec. "Results: Graphene
Nanoribbon"); those matrices are not available here, so random blocks with
the same structure stand in for them:

* lead blocks H00 (Hermitian, eigenvalues uniform in [-4, 4] eV), H01
  (complex Gaussian, spectral norm 1 eV), S00 = I + 0.1 P (P Hermitian
  positive definite, norm 1) and S01 = 0.05 G / ||G||_2, so that the Bloch
  overlap S(k) = S00 + S01 e^{ik} + S01^H e^{-ik} stays positive definite
  (the block-tridiagonal structure is the one of Sec. "Matrix equations",
  eq. infinite_system);
* a device that either copies the lead blocks on every slab or carries its
  own blocks;
* a nodal potential V_i per slab, projected with the linear shape functions
  (Sec. "Matrix equations", extrinsic-potential matrix elements).

Random draws use numpy's PCG64 (``default_rng(seed)``) in a fixed order:
Haar unitary, eigenvalues, G(H01), X(S00), G'(S01), then device draws.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

POT_DIAG = 0
POT_LINEAR_FE = 1


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """(N(0,1) + i N(0,1)) / sqrt(2), real part drawn first."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def haar_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-distributed unitary: QR of a complex Gaussian with the phase fix."""
    z = complex_gaussian(rng, (m, m))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


@dataclass
class Lead:
    H00: np.ndarray
    H01: np.ndarray
    S00: np.ndarray
    S01: np.ndarray
    V: float = 0.0

    @property
    def m(self) -> int:
        return self.H00.shape[0]


@dataclass
class Device:
    """One transport problem: two leads, N slabs of block size m, a potential."""
    N: int
    m: int
    lead_L: Lead
    lead_R: Lead
    V: np.ndarray                       # (N,) nodal potential energy, eV
    pot_mode: int = POT_LINEAR_FE
    Hd: Optional[np.ndarray] = None     # (N, m, m) or None = copies of the left lead
    Hu: Optional[np.ndarray] = None     # (N-1, m, m)
    Sd: Optional[np.ndarray] = None
    Su: Optional[np.ndarray] = None

    @property
    def uniform(self) -> bool:
        return self.Hd is None

    def blocks(self):
        """(Hd, Hu, Sd, Su) materialised (copies of the left lead if uniform)."""
        if not self.uniform:
            return self.Hd, self.Hu, self.Sd, self.Su
        L = self.lead_L
        N = self.N
        return (np.broadcast_to(L.H00, (N,) + L.H00.shape),
                np.broadcast_to(L.H01, (N - 1,) + L.H01.shape),
                np.broadcast_to(L.S00, (N,) + L.S00.shape),
                np.broadcast_to(L.S01, (N - 1,) + L.S01.shape))


@dataclass
class Workload:
    name: str
    devices: list
    energies: list                      # one energy grid per device
    eta: float = 1e-6
    extra: dict = field(default_factory=dict)

    @property
    def device(self) -> Device:
        return self.devices[0]

    @property
    def E(self) -> np.ndarray:
        return self.energies[0]


def random_lead(rng: np.random.Generator, m: int, V: float = 0.0) -> Lead:
    """Lead blocks in the fixed draw order Q, eigenvalues, G, X, G'."""
    q = haar_unitary(rng, m)
    ev = rng.uniform(-4.0, 4.0, m)
    H00 = (q * ev[None, :]) @ q.conj().T
    H00 = 0.5 * (H00 + H00.conj().T)
    g = complex_gaussian(rng, (m, m))
    H01 = g / np.linalg.norm(g, 2)
    x = complex_gaussian(rng, (m, m))
    p = x @ x.conj().T
    p = p / np.linalg.norm(p, 2)
    S00 = np.eye(m) + 0.1 * p
    S00 = 0.5 * (S00 + S00.conj().T)
    g2 = complex_gaussian(rng, (m, m))
    S01 = 0.05 * g2 / np.linalg.norm(g2, 2)
    return Lead(H00=H00, H01=H01, S00=S00, S01=S01, V=float(V))


def low_rank_coupling_lead(rng: np.random.Generator, m: int, rank: int, V: float = 0.0) -> Lead:
    """A lead whose slab coupling reaches the next slab through `rank` < m
    directions only: H01 = A B, S01 = A B' with A of m x rank columns (so
    z S01 - H01 has rank <= rank at every z), on-site blocks as in
    random_lead (drawn first, in its order)."""
    base = random_lead(rng, m, V)
    a = complex_gaussian(rng, (m, rank))
    h = a @ complex_gaussian(rng, (rank, m))
    s = a @ complex_gaussian(rng, (rank, m))
    return Lead(H00=base.H00, H01=h / np.linalg.norm(h, 2), S00=base.S00,
                S01=0.05 * s / np.linalg.norm(s, 2), V=float(V))


def tanh_barrier(N: int, height: float, width: float, ell: float = 5.0) -> np.ndarray:
    """Smooth gate-induced barrier, centred on the device, plateau `height`."""
    i = np.arange(N, dtype=np.float64)
    c = 0.5 * (N - 1)
    return height * 0.5 * (np.tanh((i - c + 0.5 * width) / ell)
                           - np.tanh((i - c - 0.5 * width) / ell))


# --------------------------------------------------------------------------
# The five workloads.  0: tiny plain FP64; 1: headline N=200, m=64;
# 2: N=400, m=128 with band-edge energies; 3: 64 uneven devices; 4: serving.
# --------------------------------------------------------------------------

def config0() -> Workload:
    rng = np.random.default_rng(0)
    N, m = 16, 8
    lead = random_lead(rng, m)
    V = np.zeros(N)
    V[6:11] = 0.3                       # slabs 6..10 inclusive
    dev = Device(N=N, m=m, lead_L=lead, lead_R=lead, V=V, pot_mode=POT_DIAG)
    return Workload("cfg0_N16_m8", [dev], [np.linspace(-3.0, 3.0, 64)], eta=1e-6)


def config1(nE: int = 2048) -> Workload:
    rng = np.random.default_rng(1)
    N, m = 200, 64
    lead = random_lead(rng, m)
    V = tanh_barrier(N, 0.4, 60.0) + rng.normal(0.0, 0.005, N)
    dev = Device(N=N, m=m, lead_L=lead, lead_R=lead, V=V, pot_mode=POT_LINEAR_FE)
    return Workload("cfg1_N200_m64", [dev], [np.linspace(-1.5, 1.5, nE)], eta=1e-6)


def config2(band_edge_energies: Optional[np.ndarray] = None) -> Workload:
    """N=400, m=128; the 256 band-edge energies are computed elsewhere (they
    need the lead band structure) and passed in; without them only the
    3840-point uniform grid is returned."""
    rng = np.random.default_rng(2)
    N, m = 400, 128
    lead = random_lead(rng, m)
    V = tanh_barrier(N, 0.4, 120.0) + rng.normal(0.0, 0.005, N)
    dev = Device(N=N, m=m, lead_L=lead, lead_R=lead, V=V, pot_mode=POT_LINEAR_FE)
    E = np.linspace(-1.5, 1.5, 3840)
    extra = {}
    if band_edge_energies is not None:
        extra["n_band_edge"] = len(band_edge_energies)
        E = np.concatenate([E, np.asarray(band_edge_energies, dtype=np.float64)])
    return Workload("cfg2_N400_m128", [dev], [E], eta=1e-6, extra=extra)


def band_edge_offsets(n: int = 256, seed: int = 2) -> np.ndarray:
    """Signed offsets delta = +-10^U(-6,-3) eV for the band-edge energy set."""
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-6.0, -3.0, n)
    sign = np.where(rng.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0)
    return sign * mag


def _square_barrier(N: int, height: float, frac: float = 0.3) -> np.ndarray:
    V = np.zeros(N)
    w = int(round(frac * N))
    s = (N - w) // 2
    V[s:s + w] = height
    return V


def config3(n_dev: int = 64, nE: int = 256, seed: int = 3) -> Workload:
    rng = np.random.default_rng(seed)
    devices, grids = [], []
    for _ in range(n_dev):
        N = int(rng.integers(50, 401))
        m = int(rng.choice([32, 64, 96, 128]))
        h = float(rng.uniform(0.1, 0.5))
        lead = random_lead(rng, m)
        devices.append(Device(N=N, m=m, lead_L=lead, lead_R=lead,
                              V=_square_barrier(N, h), pot_mode=POT_DIAG))
        grids.append(np.linspace(-1.5, 1.5, nE))
    return Workload("cfg3_batch64", devices, grids, eta=1e-6)


# Serving workload: a pool of 8 lead sets (two per block size), energies on
# the global lattice E_k = -2 + k * 2^-11 eV restricted to [-1.5, 1.5].
SERVE_DELTA = 2.0 ** -11
SERVE_E0 = -2.0


def serving_lattice() -> np.ndarray:
    k = np.arange(0, int(round(4.0 / SERVE_DELTA)) + 1)
    E = SERVE_E0 + k * SERVE_DELTA
    return E[(E >= -1.5) & (E <= 1.5)]


def serving_lead_pool(seed: int = 4):
    rng = np.random.default_rng(seed)
    pool = []
    for m in (32, 64, 96, 128):
        for _ in range(2):
            pool.append(random_lead(rng, m))
    return pool


def serving_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 4,
                     max_requests: Optional[int] = None):
    """Poisson arrivals; each request: (t_arrival, lead-pool index, N, energy
    grid on the lattice, bias).  The right lead potential is V_R = -bias,
    rounded to the lattice spacing so that E - V_R stays on the lattice, and
    the device potential ramps linearly from 0 to V_R."""
    rng = np.random.default_rng(seed + 1000)
    lattice = serving_lattice()
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        lead_idx = int(rng.integers(0, 8))
        N = int(rng.integers(50, 401))
        nE = int(rng.integers(512, 4097))
        idx = np.unique(np.round(np.linspace(0, len(lattice) - 1, nE)).astype(np.int64))
        bias = float(rng.uniform(0.0, 0.5))
        bias = round(bias / SERVE_DELTA) * SERVE_DELTA
        out.append(dict(t=t, lead=lead_idx, N=N, E=lattice[idx], bias=bias))
        if max_requests is not None and len(out) >= max_requests:
            break
    return out


def serving_device(req: dict, pool) -> Device:
    lead = pool[req["lead"]]
    N = req["N"]
    VR = -req["bias"]
    lead_R = Lead(H00=lead.H00, H01=lead.H01, S00=lead.S00, S01=lead.S01, V=VR)
    lead_L = Lead(H00=lead.H00, H01=lead.H01, S00=lead.S00, S01=lead.S01, V=0.0)
    V = np.linspace(0.0, VR, N)
    return Device(N=N, m=lead.m, lead_L=lead_L, lead_R=lead_R, V=V,
                  pot_mode=POT_LINEAR_FE)


def small_random_device(seed: int, N: int, m: int, uniform: bool = True,
                        pot_mode: int = POT_LINEAR_FE, VL: float = 0.0,
                        VR: float = 0.0, barrier: float = 0.3,
                        same_leads: bool = True) -> Device:
    """Small devices for parity sweeps: optional own device blocks (a
    perturbed copy of the lead), optional distinct right lead, a barrier."""
    rng = np.random.default_rng(seed)
    lead_L = random_lead(rng, m, VL)
    if same_leads:
        lead_R = Lead(lead_L.H00, lead_L.H01, lead_L.S00, lead_L.S01, VR)
    else:
        lead_R = random_lead(rng, m, VR)
    V = tanh_barrier(N, barrier, max(2.0, N / 3.0), ell=max(1.0, N / 40.0))
    V = V + rng.normal(0.0, 0.005, N)
    dev = Device(N=N, m=m, lead_L=lead_L, lead_R=lead_R, V=V, pot_mode=pot_mode)
    if not uniform:
        def herm(a):
            return 0.5 * (a + np.swapaxes(a.conj(), -1, -2))
        dev.Hd = herm(lead_L.H00[None] + 0.05 * complex_gaussian(rng, (N, m, m)))
        dev.Hu = lead_L.H01[None] + 0.05 * complex_gaussian(rng, (N - 1, m, m))
        dev.Sd = herm(lead_L.S00[None] + 0.002 * complex_gaussian(rng, (N, m, m)))
        dev.Su = lead_L.S01[None] + 0.002 * complex_gaussian(rng, (N - 1, m, m))
    return dev
