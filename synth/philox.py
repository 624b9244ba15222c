"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), numpy implementation.

This module is part of the seeded synthetic-input generator.  It holds none of
the polarization arithmetic.  The same bijection is implemented for the GPU in
``synth/csrc/synth_gen.hip`` so that both sides can produce bit-identical
inputs from (counter, key) without sharing any state.

All words are unsigned 32-bit values carried in numpy uint64 arrays: the
32x32 -> 64 bit product of the Philox round then never overflows.
"""
from __future__ import annotations

import numpy as np

# Round multipliers and Weyl key increments of Philox4x32 (published constants).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

_M0 = np.uint64(PHILOX_M0)
_M1 = np.uint64(PHILOX_M1)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32(c0, c1, c2, c3, k0: int, k1: int, rounds: int = 10):
    """Apply Philox4x32-R to counters (c0..c3) under key (k0, k1).

    Counters are array-likes of values < 2**32 (broadcastable); the key is a
    pair of Python ints.  Returns four uint64 arrays holding 32-bit outputs.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 &= 0xFFFFFFFF
    k1 &= 0xFFFFFFFF
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        n0 = (p1 >> _S32) ^ c1 ^ np.uint64(k0)
        n1 = p1 & _MASK
        n2 = (p0 >> _S32) ^ c3 ^ np.uint64(k1)
        n3 = p0 & _MASK
        c0, c1, c2, c3 = n0, n1, n2, n3
    return c0, c1, c2, c3
