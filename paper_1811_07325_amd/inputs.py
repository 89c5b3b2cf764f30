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


# ---------------------------------------------------------------------------
# Counter-based generator shared with the device (serving operands).
# Philox4x32-10: Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
# easy as 1, 2, 3" (SC'11), ten rounds with the published multipliers
# 0xD2511F53, 0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85.
# ---------------------------------------------------------------------------
_M32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 counters/keys -> four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _M32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _M32
    k1 = np.asarray(k1, dtype=np.uint64) & _M32
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(0x9E3779B9)) & _M32
            k1 = (k1 + np.uint64(0xBB67AE85)) & _M32
        p0 = np.uint64(0xD2511F53) * c0
        p1 = np.uint64(0xCD9E8D57) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _M32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _M32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def philox_normal(n: int, seed: int) -> np.ndarray:
    """n x n float32 with mean 0, variance 1: for element e, the sum of twelve
    24-bit uniforms (top bits of Philox outputs for counters (e_lo, e_hi, j, 0),
    j = 0..2, key (seed_lo, seed_hi)) minus 6, times 2^-24 (Irwin-Hall)."""
    e = np.arange(n * n, dtype=np.uint64)
    lo, hi = e & _M32, e >> np.uint64(32)
    k0, k1 = np.uint64(seed) & _M32, np.uint64(seed) >> np.uint64(32)
    s = np.zeros(n * n, dtype=np.int64)
    for j in range(3):
        for w in philox4x32_10(lo, hi, np.uint64(j), np.uint64(0), k0, k1):
            s += (w >> np.uint32(8)).astype(np.int64)
    v = (s - 6 * (1 << 24)).astype(np.float32) * np.float32(1.0 / 16777216.0)
    return v.reshape(n, n)
