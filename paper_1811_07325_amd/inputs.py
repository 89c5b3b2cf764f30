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
    """n x n float32 normal(0, 1) variates, elements 4m .. 4m + 3 (row-major)
    from the Philox outputs w0..w3 for counters (m_lo, m_hi, 0, 0), key
    (seed_lo, seed_hi): pair j takes u1 = float32(w_2j + 1) 2^-32, u2 =
    float32(w_2j+1) 2^-32, radius sqrt(-2 ln u1) (float64 here) and the
    float32 angle float32(2 pi) u2, element 4m + 2j = radius x cos(angle), 4m + 2j + 1 = radius x
    sin(angle), rounded to float32 -- the device generator's steps, which it
    takes in float32 with its own log, sin, cos and sqrt: the two agree to a
    few float32 ulps of the radius."""
    count = n * n
    m = np.arange((count + 3) // 4, dtype=np.uint64)
    lo, hi = m & _M32, m >> np.uint64(32)
    k0, k1 = np.uint64(seed) & _M32, np.uint64(seed) >> np.uint64(32)
    w = [x.astype(np.uint64) for x in philox4x32_10(lo, hi, np.uint64(0), np.uint64(0), k0, k1)]
    v = np.empty(4 * m.size, dtype=np.float32)
    for j in range(2):
        u1 = (w[2 * j] + np.uint64(1)).astype(np.float32).astype(np.float64) * 2.0 ** -32
        u2 = w[2 * j + 1].astype(np.float32) * np.float32(2.0 ** -32)
        radius = np.sqrt(-2.0 * np.log(u1))
        angle = (np.float32(6.2831855) * u2).astype(np.float64)     # the binary32 angle
        v[2 * j::4] = (radius * np.cos(angle)).astype(np.float32)
        v[2 * j + 1::4] = (radius * np.sin(angle)).astype(np.float32)
    return v[:count].reshape(n, n)
