"""Seeded synthetic inputs for the TDA Liouville/Davidson path.

This package produces the *inputs* of the method only: the cell and its
plane-wave sphere, a model local potential, the occupied Kohn-Sham-like
orbitals of that potential (the paper obtains them from a DFT code), their
JADE-localised rotation (Sec. 2, Eq. wannier / Eq. spread), a synthetic PDEP
screening basis (Eq. pdep) and seeded random trial blocks.

It holds none of the arithmetic of the Liouville apply, the screened-pair
construction, the pair list or the Davidson solver: both the plain CPU
oracle (``oracle/``) and the HIP library consume what it writes, and neither
imports the other.
"""
from .cell import (  # noqa: F401
    CellSpec, Cell, diamond_sites, make_cell, spec_by_name, SPECS,
    trial_block, random_block, dipole_block, near_commuting_matrices, spin_channels,
)
