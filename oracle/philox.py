"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
as 1, 2, 3", SC 2011), written from the published definition, vectorised with
numpy on 64-bit integers.  TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper (Section 2.1) renders its corpus from deterministic random numbers,
noise included, so that a voice is a pure function of its index.  Reading used
here: a counter-based generator keyed by the seed and addressed by the global
voice index, so draws do not depend on batch size or position in a batch.

  parameter draw   key = (seed lo, seed hi), counter = (g lo, g hi, p >> 2, 0),
                   word p & 3, u = (word >> 8) * 2^-24   (exact in float32)
  noise            key = (noise_seed lo, hi), counter = (g lo, g hi, n >> 3, 1),
                   16-bit half (n & 1, low half first) of word (n >> 1) & 3
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Round multipliers and Weyl key increments of Philox4x32.
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox4x32-R bijection.

    ctr: [..., 4] unsigned 32-bit words, key: [..., 2] (broadcastable).
    Each round multiplies words 0 and 2 by the two multipliers into 64-bit
    products; the new state is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).  The
    key is advanced by the Weyl constants between rounds.
    Returns [..., 4] uint32.
    """
    c = np.asarray(ctr, dtype=np.uint64) & MASK32
    k = np.asarray(key, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = k[..., 0], k[..., 1]
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0          # < 2^64: both factors are < 2^32
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _split64(x) -> tuple[np.ndarray, np.ndarray]:
    x = np.asarray(x, dtype=np.uint64)
    return x & MASK32, x >> np.uint64(32)


def u24(word) -> np.ndarray:
    """Top 24 bits of a 32-bit word as a uniform in [0, 1 - 2^-24] (exact in float32)."""
    return (np.asarray(word, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def sample_params(seed: int, voice_ids, num_params: int = 78, tag: int = 0) -> np.ndarray:
    """Normalised parameters u[g, p] in [0, 1) for the given global voice ids.

    Section 3.3: parameters are drawn uniformly in the normalised range.
    Counter (g mod 2^32, g div 2^32, p div 4, tag): tag names the synth
    architecture (0: the default Voice), so that architectures draw
    independent streams for the same seed and index.
    Returns float64 [B, num_params] whose values are exactly representable in float32.
    """
    g = np.asarray(voice_ids, dtype=np.uint64).reshape(-1)
    glo, ghi = _split64(g)
    klo, khi = _split64(np.uint64(seed))
    nblk = (num_params + 3) // 4
    blk = np.arange(nblk, dtype=np.uint64)
    ctr = np.stack(np.broadcast_arrays(glo[:, None], ghi[:, None], blk[None, :],
                                       np.full((1, 1), tag, np.uint64)), axis=-1)
    key = np.stack([klo, khi]).astype(np.uint64)
    words = philox4x32(ctr, key)  # [B, nblk, 4]
    return u24(words.reshape(len(g), nblk * 4)[:, :num_params])


def noise_halfwords(noise_seed: int, voice_id: int, n_samples: int) -> np.ndarray:
    """16-bit noise words h(n), n < n_samples, for one voice (uint32 in [0, 65535])."""
    n = np.arange(n_samples, dtype=np.uint64)
    glo, ghi = _split64(np.uint64(voice_id))
    klo, khi = _split64(np.uint64(noise_seed))
    blocks = np.arange((n_samples + 7) // 8, dtype=np.uint64)
    ctr = np.stack(np.broadcast_arrays(np.full_like(blocks, glo), np.full_like(blocks, ghi),
                                       blocks, np.ones_like(blocks)), axis=-1)
    words = philox4x32(ctr, np.stack([klo, khi]))  # [nblk, 4]
    w = words[(n >> np.uint64(3)).astype(np.int64), ((n >> np.uint64(1)) & np.uint64(3)).astype(np.int64)]
    shift = ((n & np.uint64(1)) * np.uint64(16)).astype(np.uint64)
    return ((w.astype(np.uint64) >> shift) & np.uint64(0xFFFF)).astype(np.uint32)


def noise(noise_seed: int, voice_id: int, n_samples: int) -> np.ndarray:
    """White noise x3(n) = (h + 1/2) / 32768 - 1 in (-1, 1), float64 (exact in float32)."""
    h = noise_halfwords(noise_seed, voice_id, n_samples).astype(np.float64)
    return (h + 0.5) / 32768.0 - 1.0
