"""Counter-based Gaussian test matrix (Philox4x32-10 + Box-Muller).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two
32x32->64-bit multiplies with multipliers 0xD2511F53 and 0xCD9E8D57, key bumped
by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

Mapping used by this project (the device generator implements the same one):
  key  = (seed mod 2^32, seed div 2^32)
  entry e = i*l + j of the row-major n x l matrix uses counter q = e div 2,
  ctr  = (q mod 2^32, q div 2^32, 0, 0) -> outputs (w0, w1, w2, w3)
  u1 = ((w0 >> 5) 2^26 + (w1 >> 6) + 1) 2^-53   in (0, 1]
  u2 = ((w2 >> 5) 2^26 + (w3 >> 6)) 2^-53       in [0, 1)
  e even: sqrt(-2 ln u1) cos(2 pi u2);  e odd: sqrt(-2 ln u1) sin(2 pi u2)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (uint32 values), key: 2 scalars/arrays.  Returns 4 uint64 arrays
    holding the 32-bit outputs."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for rnd in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
        if rnd < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def gaussian_philox(seed: int, n: int, ell: int) -> np.ndarray:
    total = n * ell
    npair = (total + 1) // 2
    q = np.arange(npair, dtype=np.uint64)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    w0, w1, w2, w3 = philox4x32_10((q & MASK, q >> np.uint64(32), np.zeros_like(q), np.zeros_like(q)), key)
    a1 = (w0 >> np.uint64(5)).astype(np.float64) * 67108864.0 + (w1 >> np.uint64(6)).astype(np.float64)
    a2 = (w2 >> np.uint64(5)).astype(np.float64) * 67108864.0 + (w3 >> np.uint64(6)).astype(np.float64)
    u1 = (a1 + 1.0) * 2.0 ** -53
    u2 = a2 * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty(2 * npair, dtype=np.float64)
    out[0::2] = rad * np.cos(2.0 * np.pi * u2)
    out[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return out[:total].reshape(n, ell)
