"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from the published description.

Each of the 10 rounds multiplies counter words 0 and 2 by the two round
multipliers, takes the 64-bit products' high and low halves, and permutes/XORs
them with the other two words and the key; the key is bumped by the two Weyl
constants between rounds.

Stream conventions used throughout PTSBE (the paper leaves the generator open):
  key   = (lo32(seed), hi32(seed) XOR (tag * 0x9E3779B9 mod 2^32))
  tag   = 1 for trajectory pre-sampling, 2 for shot draws, 3 for extra draws
  u     = (((w1 << 32) | w0) >> 11) * 2^-53   in [0, 1)
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)

TAG_PTS = 1
TAG_SHOTS = 2
TAG_EXTRA = 3


def key_from_seed(seed: int, tag: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    k0 = seed & 0xFFFFFFFF
    k1 = ((seed >> 32) ^ ((tag * 0x9E3779B9) & 0xFFFFFFFF)) & 0xFFFFFFFF
    return k0, k1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised over numpy arrays of counter words (values < 2^32)."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK
    c1 = np.asarray(c1, dtype=np.uint64) & MASK
    c2 = np.asarray(c2, dtype=np.uint64) & MASK
    c3 = np.asarray(c3, dtype=np.uint64) & MASK
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def uniform(seed: int, tag: int, c0, c1, c2, c3=0):
    """u in [0,1) from the top 53 bits of the first two output words."""
    k0, k1 = key_from_seed(seed, tag)
    w0, w1, _, _ = philox4x32_10(c0, c1, c2, c3, k0, k1)
    v = (w1 << np.uint64(32)) | w0
    return (v >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
