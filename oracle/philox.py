"""Philox4x64-10, written from its published definition (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
Test infrastructure only.

One block maps a 256-bit counter (4 x uint64) and a 128-bit key (2 x uint64)
to 4 x uint64 through 10 rounds.  Each round multiplies words 0 and 2 by the
two Philox multipliers (128-bit products split into hi/lo), XORs the high
halves with the other words and the key, and permutes; the key is bumped by
the two Weyl constants between rounds.

Uniforms: u = (x >> 11) * 2^-53 from word 0, i.e. the top 53 bits.
"""
from __future__ import annotations

MASK = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B


def _mulhilo(a: int, b: int):
    p = a * b
    return (p >> 64) & MASK, p & MASK


def philox4x64_10(counter, key):
    c0, c1, c2, c3 = (int(x) & MASK for x in counter)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform(seed: int, stream: int, walker: int, sweep: int, spin: int) -> float:
    """Acceptance uniform for one proposal: key (seed, stream), counter
    (walker, sweep, spin, 0)."""
    x = philox4x64_10((walker, sweep, spin, 0), (seed, stream))[0]
    return (x >> 11) * (1.0 / 9007199254740992.0)
