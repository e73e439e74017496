"""Philox4x32-10 counter-based generator.  TEST INFRASTRUCTURE ONLY.

Written from the published description (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4): a 4 x 32-bit
counter and a 2 x 32-bit key; each of the 10 rounds multiplies counter words
0 and 2 by two fixed 32-bit constants into 64-bit products, swaps and
xors the halves with the other two words and the round key, and the key is
bumped by two Weyl constants between rounds.

Pinned by the known-answer vectors of the reference distribution of that
paper (tests/golden/philox4x32_10_kat.txt).

Mapping to uniforms used by the sampler: word -> (word >> 8) * 2^-24, an
exactly representable float32 in [0, 1).  The uniform for position i of
sample b of instance q at training step t uses counter
(i // 4, b, t, q) and key (seed & 0xffffffff, seed >> 32), word i % 4.
"""

from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr [..., 4] uint32, key [..., 2] uint32 -> [..., 4] uint32."""
    c = [np.asarray(ctr[..., i], np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], np.uint64)
    k1 = np.asarray(key[..., 1], np.uint64)
    for r in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [(hi1 ^ c[1] ^ k0) & _MASK, lo1, (hi0 ^ c[3] ^ k1) & _MASK, lo0]
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def sampler_uniforms(seed: int, step: int, inst_index: int, B: int,
                     n: int) -> np.ndarray:
    """Uniforms [B, n] float32 for one instance at one training step."""
    nb = (n + 3) // 4
    b = np.arange(B, dtype=np.uint64)[:, None]
    blk = np.arange(nb, dtype=np.uint64)[None, :]
    ctr = np.zeros((B, nb, 4), np.uint64)
    ctr[..., 0] = blk
    ctr[..., 1] = b
    ctr[..., 2] = np.uint64(step & 0xFFFFFFFF)
    ctr[..., 3] = np.uint64(inst_index & 0xFFFFFFFF)
    key = np.zeros((B, nb, 2), np.uint64)
    key[..., 0] = np.uint64(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint64((seed >> 32) & 0xFFFFFFFF)
    words = philox4x32_10(ctr, key).reshape(B, nb * 4)[:, :n]
    return ((words >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
