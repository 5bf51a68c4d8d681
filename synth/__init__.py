"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only *draws* inputs: the spring-network glass whose unweighted
3x3 force-constant blocks and masses define the vibrational problem, and seeded
Gaussian start blocks.  It holds none of the eigensolver's arithmetic (no mass
weighting, no spectral map, no filter): both the HIP library and the CPU oracle
consume these arrays and do the method's work on their own.
"""
from .glass import Glass, lattice_glass, offdiag_count, relabel
from .vectors import gaussian_block, gaussian_vector

__all__ = ["Glass", "lattice_glass", "offdiag_count", "relabel", "gaussian_block", "gaussian_vector"]
