"""ORACLE (test infrastructure): Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the
published definition: ten rounds of two 32x32->64-bit multiplications by the
constants 0xD2511F53 and 0xCD9E8D57, with the Weyl key schedule
(0x9E3779B9, 0xBB67AE85) added to the key before every round after the first.

Use in the sampler: key = seed (low word, high word); counter =
(low word of the stream index, high word, draw id, 0); one 53-bit uniform
U = ((w1 << 32 | w0) >> 11) * 2^-53 from the first two output words.

Everything is vectorised over NumPy uint64 arrays holding 32-bit values.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k = [np.asarray(k0, dtype=np.uint64) & MASK, np.asarray(k1, dtype=np.uint64) & MASK]
    for r in range(10):
        if r > 0:
            k = [(k[0] + W0) & MASK, (k[1] + W1) & MASK]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


def uniform53(seed: int, stream, draw_id: int) -> np.ndarray:
    """U in [0, 1) for each 64-bit stream index (array-like), as float64."""
    stream = np.asarray(stream, dtype=np.uint64)
    seed = np.uint64(seed)
    w = philox4x32_10(stream & MASK, stream >> S32, np.uint64(draw_id), np.uint64(0),
                      seed & MASK, seed >> S32)
    x = (w[1] << S32) | w[0]
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def raw64(seed: int, stream, draw_id: int) -> np.ndarray:
    stream = np.asarray(stream, dtype=np.uint64)
    seed = np.uint64(seed)
    w = philox4x32_10(stream & MASK, stream >> S32, np.uint64(draw_id), np.uint64(0),
                      seed & MASK, seed >> S32)
    return (w[1] << S32) | w[0]
