"""Writes cfg2_band_edge_energies.txt: 256 energies within 1 meV of the band
extrema of the N = 400, m = 128 workload's lead.

The extrema are those of the lead's complex bands E_n(k) from the Bloch
eigenproblem H(k) c = E S(k) c (Sec. "Electronic Structure"), found by the
oracle (a 4096-point k scan, then Brent's method on the Hellmann-Feynman
slope to 1e-12 in k); only extrema inside [-1.5, 1.5] eV are used.  Energy
k of the set is edge[floor(k n_edges / 256)] + delta_k (extrema spread
evenly over the sorted list) with the seeded offsets
delta = +-10^U(-6,-3) eV of the workload generator.  Calls only the oracle
(and the seeded input generator for the lead blocks).

    python tests/golden/make_band_edges.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bands                      # noqa: E402
from paper_1903_00548_amd import workloads    # noqa: E402


def main():
    lead = workloads.config2().device.lead_L
    edges = bands.band_extrema(lead.H00, lead.H01, lead.S00, lead.S01, 0.0, nk=4096, window=(-1.5, 1.5))
    delta = workloads.band_edge_offsets(256)
    # extrema taken evenly over the sorted list (all of them, cyclically, when
    # there are fewer extrema than energies)
    n = len(edges)
    pick = [(k * n) // len(delta) if n >= len(delta) else k % n for k in range(len(delta))]
    E = np.array([edges[p] + delta[k] for k, p in enumerate(pick)])
    out = os.path.join(HERE, "cfg2_band_edge_energies.txt")
    with open(out, "w") as f:
        f.write("# 256 energies (eV) within 1 meV of the lead band extrema of the N=400, m=128 workload\n")
        f.write(f"# {len(edges)} extrema in [-1.5, 1.5] eV; written by tests/golden/make_band_edges.py\n")
        for e in E:
            f.write(f"{e:.17g}\n")
    print(f"{len(edges)} extrema, wrote {out}")


if __name__ == "__main__":
    main()
