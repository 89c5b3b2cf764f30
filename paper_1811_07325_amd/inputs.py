"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the Strassen method: it only draws matrices.
The paper multiplies random double-precision matrices (Section V-A); these
generators stand in for them with stated distributions and seeds:

* ``uniform(n, seed)``  -- i.i.d. uniform[-1, 1], float32 (PCG64).
* ``integers(n, seed)`` -- i.i.d. integers uniform in [lo, hi], stored as float32.
* ``normal(n, seed)``   -- i.i.d. normal(0, 1), float32 (PCG64).
* ``sample_rows``/``gaussian_vector`` -- seeded row samples and probe vectors.
"""
from __future__ import annotations

import numpy as np


def uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, n)).astype(np.float32)


def integers(n: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, n)).astype(np.float32)


def normal(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(n, n), dtype=np.float32)


def sample_rows(n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct row indices of an n x n matrix, sorted."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=n)  # float64
