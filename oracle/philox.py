"""Philox4x32-10 counter-based generator (test oracle).

Written from the published definition: J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
SC'11, Section 5 (the Philox S-box).  A 128-bit counter (c0, c1, c2, c3)
and a 64-bit key (k0, k1) go through 10 rounds.  One round multiplies c0
and c2 by two fixed odd 32-bit constants, keeping the high and low halves
of each 64-bit product, and forms

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0));

between rounds the key is advanced by two Weyl constants (the golden ratio
and sqrt(3) - 1 scaled to 32 bits).  The paper this project implements does
not fix a generator; Philox is this project's choice for reproducible,
counter-addressable Monte Carlo frames.

Vectorised over NumPy uint64 arrays holding 32-bit values.  Pinned against
rocRAND's independent implementation (run as a library on the host).
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
MUL0 = np.uint64(0xD2511F53)
MUL1 = np.uint64(0xCD9E8D57)
WEYL0 = np.uint64(0x9E3779B9)
WEYL1 = np.uint64(0xBB67AE85)
ROUNDS = 10


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = ROUNDS):
    """Return the four 32-bit output words (as uint64 arrays)."""
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & MASK32
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + WEYL0) & MASK32
            k1 = (k1 + WEYL1) & MASK32
        p0 = MUL0 * c0  # < 2^64, exact in uint64
        p1 = MUL1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
