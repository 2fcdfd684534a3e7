"""Philox-4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition.

TEST INFRASTRUCTURE ONLY (see the package header).

One round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
    (hi(B * c2) ^ c1 ^ k0,  lo(B * c2),  hi(A * c0) ^ c3 ^ k1,  lo(A * c0))
with A = 0xD2511F53, B = 0xCD9E8D57 and hi / lo the upper and lower 32 bits
of the 64-bit product; the key is advanced by the Weyl constants
(0x9E3779B9, 0xBB67AE85) after each of the ten rounds.

The sampler's uniforms take the top 24 bits of the first output word:
u = (x >> 8) / 2^24, so u lies in [0, 1) and is exact in FP32.

Parity: pinned by the known-answer vectors published with the generator
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np

_A = np.uint64(0xD2511F53)
_B = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: array (..., 4) of uint32 values, key: (k0, k1).  Returns (..., 4)
    uint64 arrays holding the 32-bit outputs."""
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _A * c0                  # < 2^64: both factors are below 2^32
        p1 = _B * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0)
        n1 = p1 & _MASK
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1)
        n3 = p0 & _MASK
        c0, c1, c2, c3 = n0, n1, n2, n3
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack([c0, c1, c2, c3], axis=-1)


def site_uniforms(shots, site: int, seed: int) -> np.ndarray:
    """u for each shot index in `shots` at `site` (1-based): counter
    (shot low word, shot high word, site, 0), key (seed low word, seed high
    word), first output word, top 24 bits."""
    s = np.asarray(shots, dtype=np.uint64)
    ctr = np.stack([s & _MASK, s >> np.uint64(32), np.full_like(s, site), np.zeros_like(s)], axis=-1)
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))[..., 0]
    return (x >> np.uint64(8)).astype(np.float64) / 16777216.0
