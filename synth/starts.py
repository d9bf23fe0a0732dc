"""Seeded start vectors.

The paper leaves x_init open (Algorithm 1 takes it as an input). Starts are
drawn here, from numpy's PCG64 generator, and handed to both the oracle and
the GPU path as data, so the two sides never draw random numbers themselves.
"""

from __future__ import annotations

import numpy as np


def start_vector(n: int, seed: int) -> np.ndarray:
    """Standard-normal float64 vector of length n (not normalised)."""
    return np.random.default_rng(seed).standard_normal(n)


def start_block(n: int, k: int, seed: int) -> np.ndarray:
    """k independent standard-normal starts, shape (k, n), row s is start s."""
    return np.random.default_rng(seed).standard_normal((k, n))
