"""Oracle of the noise step (test infrastructure; not imported by the product path).

The paper's pipeline ends by adding realistic noise (arXiv:2412.08265, Sec. 3) without giving a
model. Reading taken here: every voxel of the final cube gets independent Gaussian noise of
variance  gain * max(C, 0) + sigma_floor^2  (a photon term in the Gaussian limit plus a floor).

The normal deviates come from a counter-based generator so that any implementation draws the
same numbers: Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011), key (seed_lo, seed_hi), counter (voxel_lo, voxel_hi, stream, 0).
Of its four 32-bit outputs x0, x1 the first two give u = (x + 1/2) 2^-32 in (0, 1), and the
Box-Muller transform eps = sqrt(-2 ln u0) cos(2 pi u1) (FP64) a standard normal deviate.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Philox-4x32 multipliers and Weyl key increments as published
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays of uint32 values (as uint64), key: (k0, k1). Returns 4 uint64 arrays of
    32-bit outputs. One round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key gains (W0, W1) between rounds."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr)
    k0, k1 = np.uint64(key[0]) & MASK32, np.uint64(key[1]) & MASK32
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0                      # < 2^64: exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def normals(n: int, seed: int, stream: int) -> np.ndarray:
    """Standard normal deviates for voxels 0..n-1 of one stream, FP64."""
    i = np.arange(n, dtype=np.uint64)
    x0, x1, _, _ = philox4x32_10((i & MASK32, i >> np.uint64(32), np.full(n, stream, np.uint64),
                                  np.zeros(n, np.uint64)),
                                 (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u0 = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
    u1 = (x1.astype(np.float64) + 0.5) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def add_noise(cube: np.ndarray, seed: int, stream: int, gain: float,
              sigma_floor: float) -> np.ndarray:
    """cube + sqrt(gain max(cube, 0) + sigma_floor^2) eps, voxel v in C order, FP64."""
    c = np.asarray(cube, dtype=np.float64)
    eps = normals(c.size, seed, stream).reshape(c.shape)
    return c + np.sqrt(gain * np.maximum(c, 0.0) + sigma_floor * sigma_floor) * eps
