"""Philox4x32-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE: part of the CPU oracle; only tests, the smoke check and
the benchmark's CPU-baseline leg may import it.

Definition (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Sec. 3.3 "Philox"): a 4-word counter (c0, c1, c2, c3) and a
2-word key (k0, k1) of 32-bit words go through R = 10 rounds.  One round
multiplies c0 and c2 by the constants M0 = 0xD2511F53 and M1 = 0xCD9E8D57 as
32x32 -> 64-bit products and returns

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)).

Between consecutive rounds the key is advanced by the Weyl constants
W0 = 0x9E3779B9 and W1 = 0xBB67AE85 (mod 2^32).  The method draws its random
numbers from this generator; the stream layout (which counter word carries
what) is defined in ``oracle.mpr``.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SHIFT32 = np.uint64(32)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Return the four 32-bit output words for the given counters and key.

    All arguments broadcast against each other; they are taken modulo 2^32.
    The outputs are numpy uint32 arrays of the broadcast shape.
    """
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & MASK32
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0            # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> SHIFT32, p0 & MASK32
        hi1, lo1 = p1 >> SHIFT32, p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(w.astype(np.uint32) for w in (c0, c1, c2, c3))


def unit_float(w):
    """Map a 32-bit word to [0, 1 - 2^-24] as (w >> 8) * 2^-24.

    The result has 24 significant bits, so it is exact in both float32 and
    float64 and both precisions consume the identical number.
    """
    return (np.asarray(w, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
