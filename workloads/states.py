"""Seeded random population deviations (inputs only)."""

import numpy as np


def random_deviations(q: int, n: int, seed: int, amp: float = 1e-3) -> np.ndarray:
    """Deviations delta[i, s] ~ U(-amp, amp), float64 [q, n].

    A state f_i = w_i + delta_i stays positive for amp below the smallest
    lattice weight; nothing here depends on the lattice beyond its size.
    """
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(q, n))
