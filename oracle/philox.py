"""Philox-4x32-10 and the seeded draws of an instance, in plain numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper leaves the random draws of its generator open (random permutation
P, random supports and values, section 4.1 and Procedure OsGen, section 6).
Both the HIP library and this oracle take every such draw from one
counter-based generator, Philox-4x32-10, defined in

    J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
    numbers: as easy as 1, 2, 3", SC'11 (section 3 and Table 2).

Each side implements it on its own from that definition.  All arithmetic
here is on numpy uint64 arrays that hold 32-bit values, so products of two
32-bit words are exact.
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Multipliers and Weyl key increments of Philox-4x32 (Salmon et al., Table 2).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def _u64(a):
    return np.asarray(a, dtype=np.uint64) & MASK32


def philox4x32_10(c0, c1, c2, c3, key):
    """Ten rounds of Philox-4x32 on counter (c0,c1,c2,c3) under key (k0,k1).

    One round: the products M0*c0 and M1*c2 are split into high and low
    words; the new counter is (hi1^c1^k0, lo1, hi0^c3^k1, lo0).  The key is
    advanced by the Weyl constants before every round after the first.
    Returns four uint64 arrays holding 32-bit words.
    """
    c0, c1, c2, c3 = (_u64(c) for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def seed_key(seed):
    """Philox key of an instance seed: its low and high 32-bit halves."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def unit_double(lo, hi):
    """Uniform double in [0,1) from two 32-bit words: top 53 bits of hi:lo."""
    w = (_u64(hi) << np.uint64(32)) | _u64(lo)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
