"""Gaussian test tensor drawn from a counter-based generator, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 6 draws Gaussian tensor columns G ("generate a Gaussian random tensor").  To compare a
factorization whose Gaussian tensor was drawn on the device with the oracle's, both sides
implement one published generator, each from its definition (nothing shared):

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
  SC 2011): a 4 x 32-bit counter and a 2 x 32-bit key; each of the ten rounds multiplies counter
  words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 (full 64-bit products), and the new counter is
  (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1, lo(c0 M0)); the key is then increased by
  (0x9E3779B9, 0xBB67AE85) modulo 2^32.
* Box-Muller (Box and Muller, Ann. Math. Stat. 29, 1958): two independent uniforms u1 in (0, 1],
  u2 in [0, 1) give two independent standard normals sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).

Layout of the m x r x n tensor (math order, element (i, j, t)): linear index e = i + m j + m r t
(column-major, frontal slices contiguous); pair q = e // 2 uses the counter (q mod 2^32, q div 2^32,
0, 0) and the key (seed mod 2^32, seed div 2^32); its output words x0..x3 give
u1 = ((x1 x0 >> 11) + 1/2) 2^-53 and u2 = (x3 x2 >> 11) 2^-53 (64-bit words high:low); element 2q is
the cosine term, element 2q + 1 the sine term.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)


def philox4x32_10(counter, key):
    """Philox4x32-10 of the counters (4 arrays of 32-bit words) under the key (2 words).

    Returns the four output words as uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK for c in counter)
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    for _ in range(10):
        p0 = c0 * _M0            # both factors < 2^32: exact in 64 bits
        p1 = c2 * _M1
        c0, c1, c2, c3 = (((p1 >> np.uint64(32)) ^ c1 ^ k0) & _MASK, p1 & _MASK,
                          ((p0 >> np.uint64(32)) ^ c3 ^ k1) & _MASK, p0 & _MASK)
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def normal_pairs(seed: int, q: np.ndarray):
    """The two standard normals of pair indices q (Box-Muller on Philox4x32-10 output)."""
    q = np.asarray(q, dtype=np.uint64)
    zero = np.zeros_like(q)
    seed = int(seed) & ((1 << 64) - 1)
    x0, x1, x2, x3 = philox4x32_10((q & _MASK, q >> np.uint64(32), zero, zero), (seed & 0xFFFFFFFF, seed >> 32))
    a = ((x1 << np.uint64(32)) | x0) >> np.uint64(11)
    b = ((x3 << np.uint64(32)) | x2) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2)


def gaussian_tensor(seed: int, m: int, r: int, n: int) -> np.ndarray:
    """The m x r x n Gaussian tensor of the layout above, math order (m, r, n), float64."""
    count = m * r * n
    q = np.arange((count + 1) // 2, dtype=np.uint64)
    z0, z1 = normal_pairs(seed, q)
    flat = np.empty(2 * q.size)
    flat[0::2] = z0
    flat[1::2] = z1
    # linear index e = i + m j + m r t  ->  column-major (m, r, n)
    return flat[:count].reshape((m, r, n), order="F")
