"""CPU reference (oracle) for the closed-shell in-situ (T) energy.

TEST INFRASTRUCTURE, NOT PART OF THE LIBRARY.  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import or run anything here; the
library never does, and this package imports nothing from the library.

Everything is plain float64 numpy written from the paper's section on the
in-situ form of perturbative (T) in SIE (equation E_corr_CCSD_T and the W, V,
D, W-tilde, P, R and C^f definitions that follow it), plus an independent
spin-orbital evaluation of the textbook (T) formula used as a pin.

Pinned by tests/test_oracle_pins.py; see the module docstrings for which
function each pin covers.
"""

from .triples import (  # noqa: F401
    energy_literal,
    energy_literal_vectorized,
    energy_dense,
    projector_matrix,
    occupied_triple_energy,
    occupied_triple_parts,
    energy_by_occupied_triples,
    occupied_triples,
    triple_weight,
    flops_per_fragment,
)
from .spinorb import spin_orbital_triples, mp4_triples_ordered  # noqa: F401
