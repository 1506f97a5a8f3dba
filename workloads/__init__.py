"""Seeded, synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This package only *builds inputs*: node-type maps of 2D fibre cross-sections,
per-node catalytic rates, and the lattice parameters that correspond to a
(Pe, Da) pair.  It holds none of the lattice-Boltzmann arithmetic and imports
neither the GPU binding nor the oracle.
"""
from .geometry import (FLUID, SOLID, CAT1, CAT2, channel, disc_offsets, place_discs,
                       rasterize, classify_surface, surface_counts)
from .configs import (U0, TAU_F, LatticeParams, lattice_params, Workload, make_workload,
                      CONFIGS, batch_instances, box_workload)

__all__ = [
    "FLUID", "SOLID", "CAT1", "CAT2", "channel", "disc_offsets", "place_discs", "rasterize",
    "classify_surface", "surface_counts", "U0", "TAU_F", "LatticeParams", "lattice_params",
    "Workload", "make_workload", "CONFIGS", "batch_instances", "box_workload",
]
