"""Seeded Gaussian start blocks and probe vectors (numpy PCG64)."""
from __future__ import annotations

import numpy as np


def gaussian_block(n: int, q: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Row-major [n][q] block of independent standard normal entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((n, q)).astype(dtype, copy=False))


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)
