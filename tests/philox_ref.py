"""Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011), written from its definition for the tests: ten
rounds of two 32x32->64-bit multiplications by 0xD2511F53 and 0xCD9E8D57 with
the key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
The library's start points are checked against this reference, and this
reference against the generator's published known-answer vectors."""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
    return c0, c1, c2, c3


def philox_first_words(ctr0, ctr1, key, ctr2=0):
    """First output word for counters (ctr0[i], ctr1[i], ctr2, 0), vectorised over
    numpy uint64 arrays holding 32-bit values."""
    c0 = np.asarray(ctr0, dtype=np.uint64) & MASK
    c1 = np.asarray(ctr1, dtype=np.uint64) & MASK
    c2 = np.full_like(c0, int(ctr2) & MASK)
    c3 = np.zeros_like(c0)
    k0, k1 = np.uint64(int(key[0]) & MASK), np.uint64(int(key[1]) & MASK)
    m = np.uint64(MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
        p0 = np.uint64(M0) * c0          # < 2^64: no wrap
        p1 = np.uint64(M1) * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0) & m, p1 & m, ((p0 >> np.uint64(32)) ^ c3 ^ k1) & m, p0 & m
    return c0


def uniform_pm1(words):
    """Top 24 bits u of a 32-bit word -> u * 2^-23 - 1, exact in FP32."""
    u = (np.asarray(words, dtype=np.uint64) & np.uint64(MASK)) >> np.uint64(8)
    return (u.astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)
