"""Seeded spin batches, ``int8`` values in {-1, +1} (s = 2x - 1 for occupation x)."""
from __future__ import annotations

import numpy as np


def random_sz0_spins(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """``batch`` independent uniform configurations with zero total S_z (N/2 up spins)."""
    if n_sites % 2:
        raise ValueError("S_z = 0 needs an even number of sites")
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = rng.random((batch, n_sites))
    rank = np.argsort(np.argsort(keys, axis=1), axis=1)
    return np.where(rank < n_sites // 2, 1, -1).astype(np.int8)


def random_spins(batch: int, n_sites: int, seed: int) -> np.ndarray:
    """Unconstrained uniform spins (any S_z), for edge cases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.where(rng.random((batch, n_sites)) < 0.5, 1, -1).astype(np.int8)
