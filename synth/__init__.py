"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only *draws* inputs: water-like orbital sets built from periodic
Gaussians on a real-space grid.  It holds none of the exchange method's
arithmetic (no FFT, no Poisson kernel, no localization, no ACE algebra).
"""
from .orbitals import (  # noqa: F401
    SystemSpec, OrbitalSet, CONFIGS, config_spec, batched_specs, training_specs, batched_like_specs,
    make_orbitals, smooth_test_vectors, lattice_dims, box_length_for, disjoint_gaussians, make_bloch_orbitals,
)
