"""Philox4x32-10 counter-based generator and Box-Muller white noise (FP64).

Test infrastructure only (see ``oracle/__init__``).

The initial-condition generator of Sec. 2.3.2 multiplies a Gaussian random field by the
transfer function. The Gaussian numbers it draws cannot be handed in from outside at the
largest sizes, so each side implements the same counter-based generator from its published
definition: Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random
numbers: as easy as 1, 2, 3").

Stream definition used here: lattice point with linear index i (x fastest) and 64-bit seed s
uses counter (i mod 2^32, i >> 32, 0, 0) and key (s mod 2^32, s >> 32). Outputs r0, r1 give
u_j = (r_j + 1/2) 2^-32 in (0, 1) and the normal deviate
    w = sqrt(-2 ln u_0) cos(2 pi u_1).

Pins (tests/test_oracle_rng.py): the known-answer vectors published with the Random123
distribution; sample moments of w.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10. ctr: (..., 4) uint32-valued, key: (..., 2). Returns (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & _MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def white_noise(seed: int, n: int, start: int = 0, count: int | None = None) -> np.ndarray:
    """Unit-variance Gaussian white noise for lattice indices start .. start+count-1 (FP64)."""
    if count is None:
        count = n**3 - start
    idx = np.arange(start, start + count, dtype=np.uint64)
    ctr = np.zeros((count, 4), dtype=np.uint64)
    ctr[:, 0] = idx & _MASK
    ctr[:, 1] = idx >> np.uint64(32)
    key = np.zeros((count, 2), dtype=np.uint64)
    key[:, 0] = np.uint64(seed) & _MASK
    key[:, 1] = np.uint64(seed) >> np.uint64(32)
    r = philox4x32_10(ctr, key)
    u0 = (r[:, 0].astype(np.float64) + 0.5) * 2.0**-32
    u1 = (r[:, 1].astype(np.float64) + 0.5) * 2.0**-32
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def white_noise_grid(seed: int, n: int) -> np.ndarray:
    """Noise on the n^3 lattice as an array indexed [z, y, x]."""
    return white_noise(seed, n).reshape(n, n, n)
