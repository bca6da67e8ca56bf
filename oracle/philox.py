"""Philox4x32-10 counter-based generator and the Gaussian sketch it defines.

Philox is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  One round maps a
4-word counter (c0, c1, c2, c3) under a 2-word key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with M0 = 0xD2511F53 and M1 = 0xCD9E8D57 (32x32 -> 64-bit products split into
high and low words).  Between rounds the key is bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85).  Ten rounds.

Gaussian sketch (Algorithm 2, Phase 1: Omega with i.i.d. N(0,1) entries,
Assumption 1.5).  Entry (i, k) of the n x w sketch for seed s:

    counter = (i mod 2^32, i >> 32, k >> 1, 0),  key = (s mod 2^32, s >> 32)
    (o0, o1, o2, o3) = Philox(counter, key)
    u1 = ((o0 << 32 | o1) >> 11) * 2^-53 + 2^-54       (in (0, 1))
    u2 = ((o2 << 32 | o3) >> 11) * 2^-53 + 2^-54
    rad = sqrt(-2 ln u1)
    Omega[i, k] = rad * cos(2 pi u2)  if k even,  rad * sin(2 pi u2)  if k odd

(Box-Muller transform, Box and Muller 1958.)  This module is written from
that definition independently of the GPU library.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: uint32-valued array of shape (4, N); key: shape (2, N) or (2,).
    Returns a (4, N) uint64 array holding 32-bit outputs.
    """
    c = [np.asarray(ctr[i], dtype=np.uint64) & MASK for i in range(4)]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]  # < 2^64, exact in uint64
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c)


def _uniform53(hi, lo):
    x = (hi << np.uint64(32)) | lo
    return (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 + 2.0 ** -54


def gaussian_sketch(n: int, w: int, seed: int) -> np.ndarray:
    """The n x w Philox/Box-Muller sketch defined above (row-major array)."""
    seed = int(seed)
    rows = np.arange(n, dtype=np.uint64)
    pairs = (w + 1) // 2
    out = np.empty((n, 2 * pairs), dtype=np.float64)
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    for kp in range(pairs):
        ctr = (rows & MASK, rows >> np.uint64(32),
               np.full(n, kp, dtype=np.uint64), np.zeros(n, dtype=np.uint64))
        o = philox4x32_10(ctr, key)
        u1 = _uniform53(o[0], o[1])
        u2 = _uniform53(o[2], o[3])
        rad = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * kp] = rad * np.cos(2.0 * np.pi * u2)
        out[:, 2 * kp + 1] = rad * np.sin(2.0 * np.pi * u2)
    return out[:, :w].copy()
