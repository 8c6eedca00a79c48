"""Plain, slow FP64 CPU oracle for the open-boundary transport solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path.

What it computes, per energy E (z = E + i eta, applied in the leads and the
device alike):

* lead self-energies from the complex band structure of each contact, by
  the symmetric linearisation of the quadratic eigenvalue problem and the
  Bloch-matrix projection (Sec. "Contact self-energies",
  eqs. complex_bs and linearized_eigenvalue_symmetric, and the Sigma = [H' -
  E M'] B Lambda B^-1 formula that follows them);
* the Green's-function columns of the block-tridiagonal open system
  (Sec. "Extended states", eq. qtbm_system and the NEGF paragraph after it);
* transmission T(E) = Re Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H] and the
  slab-resolved density of states per injecting contact
  n_i = (1/pi) Re sum_{j in slab i} [G Gamma G^H]_jj (Sec. "Density", node
  density; Sec. "Transmission and Ballistic Current");
* the nearest-neighbour blocks of the slab-basis density matrix over an
  energy grid with per-contact weights (Sec. "Density",
  eq. density_matrices; oracle.density_matrix);
* the paper's own mode-space QTBM at eta = 0 as a cross-check (eqs.
  hellmann-feynman, normalization, transmission).

Pins: closed-form 1-band barrier transmission, integer transmission of a
perfect lead-identical wire, T + R = number of open modes, dense brute-force
inversion on tiny systems, an independent decimation and a brute-force
finite lead for the self-energy.  All are in tests/test_oracle_*.py.
"""
from .leads import (lead_operators, complex_band_modes, self_energies,
                    broadening, open_channels)
from .device import (potential_weights, assemble, first_block_column,
                     last_block_column, columns_dense, columns_banded,
                     columns_two_pass)
from .observables import transmission, slab_dos, solve_energy, solve_device
from .density_matrix import density_matrix_blocks

__all__ = [
    "lead_operators", "complex_band_modes", "self_energies", "broadening",
    "open_channels", "potential_weights", "assemble", "first_block_column",
    "last_block_column", "columns_dense", "columns_banded", "columns_two_pass",
    "transmission", "slab_dos", "solve_energy", "solve_device",
    "density_matrix_blocks",
]
