"""Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011) and the seeded feature-map draw built on it, in
NumPy, written from the published definition for the tests: ten rounds of
two 32 x 32 -> 64-bit products by M0 = 0xD2511F53 and M1 = 0xCD9E8D57, the
high halves XORed with the other two counter words and the round key, the
key advanced by the Weyl increments 0x9E3779B9, 0xBB67AE85 after each round.
Independent of the library's device code."""

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, key):
    """Vectorised over counter arrays (uint32 values); key = (k0, k1)."""
    x = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0, k1 = key[0] & 0xFFFFFFFF, key[1] & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        x = [hi1 ^ x[1] ^ np.uint64(k0), lo1, hi0 ^ x[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return x


def _uniform(hi, lo):
    v = (hi << np.uint64(32)) | lo
    return ((v >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def draw_features(seed, d, s, sigma):
    """(W d x s, b s) float32 as documented with bsadmm_problem.seed."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    count = d * s
    t = np.arange((count + 1) // 2, dtype=np.uint64)
    w = philox4x32_10(t & MASK, t >> np.uint64(32), np.zeros_like(t), np.zeros_like(t), key)
    u1, u2 = _uniform(w[0], w[1]), _uniform(w[2], w[3])
    r = np.sqrt(-2.0 * np.log(u1)) / sigma
    z = np.empty(2 * t.size, dtype=np.float64)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    W = z[:count].astype(np.float32).reshape(d, s)
    j = np.arange(s, dtype=np.uint64)
    w = philox4x32_10(j & MASK, j >> np.uint64(32), np.ones_like(j), np.zeros_like(j), key)
    b = (2.0 * np.pi * _uniform(w[0], w[1])).astype(np.float32)
    b[b >= np.float32(2.0 * np.pi)] = 0.0
    return W, b
