"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

Written from the published definition: a 4x32-bit counter and a 2x32-bit key
go through ten rounds; each round takes the two 32x32->64 products of the
counter words 0 and 2 with fixed multipliers, mixes the high halves with the
other counter words and the key, and the key is bumped by two Weyl constants
between rounds.

This module holds random-number generation only. It is the single source of
seeded randomness for every workload, shared by the GPU path and the oracle.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(counter, key):
    """Ten-round Philox on arrays of counters.

    counter: uint32-compatible array of shape (..., 4); key: two uint32.
    Returns uint32 array of shape (..., 4).
    """
    c = np.asarray(counter, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0 = np.uint64(int(key[0]) & 0xFFFFFFFF)
    k1 = np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0            # < 2^64, exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


class Stream:
    """A reproducible stream of doubles keyed by (seed, stream id).

    Block b of the stream is Philox(counter=(b, 0, 0, 0), key=(seed, stream)).
    Each block yields two doubles in [0, 1) with 53 random bits each.
    """

    def __init__(self, seed: int, stream: int):
        self.key = (int(seed), int(stream))
        self.block = 0

    def _words(self, nblocks: int) -> np.ndarray:
        ctr = np.zeros((nblocks, 4), dtype=np.uint64)
        ctr[:, 0] = np.arange(self.block, self.block + nblocks, dtype=np.uint64)
        self.block += nblocks
        return philox4x32(ctr, self.key)

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        nb = (n + 1) // 2
        w = self._words(nb).astype(np.uint64)
        a = (w[:, 0] >> np.uint64(5)) * np.uint64(1 << 26) + (w[:, 1] >> np.uint64(6))
        b = (w[:, 2] >> np.uint64(5)) * np.uint64(1 << 26) + (w[:, 3] >> np.uint64(6))
        u = np.stack([a, b], axis=1).reshape(-1)[:n].astype(np.float64) / float(1 << 53)
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        """Box-Muller normals."""
        m = (n + 1) // 2
        u1 = self.uniform(m)
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log1p(-u1))      # 1 - u1 in (0, 1]
        z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
        return z[:n]

    def integers(self, n: int, lo: int, hi: int) -> np.ndarray:
        """Integers uniform on [lo, hi] inclusive."""
        u = self.uniform(n)
        return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)
