"""Oracle of the noise step (test infrastructure; not imported by the product path).

The paper's pipeline ends by adding realistic noise (arXiv:2412.08265, Sec. 3) without giving a
model. Reading taken here: every voxel of the final cube gets independent Gaussian noise of
variance  gain * max(C, 0) + sigma_floor^2  (a photon term in the Gaussian limit plus a floor).

The normal deviates come from a counter-based generator so that any implementation draws the
same numbers: Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011), key (seed_lo, seed_hi), counter (b_lo, b_hi, stream, 0) for the
block b of voxels 4b .. 4b+3. Its four 32-bit outputs x0..x3 give u_k = (x_k + 1/2) 2^-32 in
(0, 1), and the Box-Muller transform (Box and Muller 1958) turns each pair (u0, u1), (u2, u3)
into two independent standard normal deviates, in FP64:
  eps(4b)   = r0 cos(2 pi u1),  eps(4b+1) = r0 sin(2 pi u1),  r0 = sqrt(-2 ln u0),
  eps(4b+2) = r1 cos(2 pi u3),  eps(4b+3) = r1 sin(2 pi u3),  r1 = sqrt(-2 ln u2).
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
    """Standard normal deviates for voxels 0..n-1 of one stream, FP64 (one Philox block per
    four voxels; the last block's unused deviates are dropped)."""
    nb = (n + 3) // 4
    b = np.arange(nb, dtype=np.uint64)
    x = philox4x32_10((b & MASK32, b >> np.uint64(32), np.full(nb, stream, np.uint64),
                       np.zeros(nb, np.uint64)),
                      (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    u = [(xk.astype(np.float64) + 0.5) * 2.0 ** -32 for xk in x]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r1 = np.sqrt(-2.0 * np.log(u[2]))
    eps = np.empty((nb, 4))
    eps[:, 0] = r0 * np.cos(2.0 * np.pi * u[1])
    eps[:, 1] = r0 * np.sin(2.0 * np.pi * u[1])
    eps[:, 2] = r1 * np.cos(2.0 * np.pi * u[3])
    eps[:, 3] = r1 * np.sin(2.0 * np.pi * u[3])
    return eps.ravel()[:n]


def add_noise(cube: np.ndarray, seed: int, stream: int, gain: float,
              sigma_floor: float) -> np.ndarray:
    """cube + sqrt(gain max(cube, 0) + sigma_floor^2) eps, voxel v in C order, FP64."""
    c = np.asarray(cube, dtype=np.float64)
    eps = normals(c.size, seed, stream).reshape(c.shape)
    return c + np.sqrt(gain * np.maximum(c, 0.0) + sigma_floor * sigma_floor) * eps
