"""Seeded channel noise and bit packing.

Code-capacity noise as used in Section IV-A: i.i.d. bit flips with
probability p per qubit, or depolarising noise (X, Y, Z each with
probability p/3).  Draws use numpy's PCG64 with a (seed, stream) key and are
produced in shot chunks so that 10^5..10^6-shot batches stay small in host
memory: each qubit compares a uniform 32-bit integer against
round(p * 2^32).

Bit packing is LSB-first: bit i of a row lives in word i // 64 at position
i % 64.  The channel LLR of a flip probability p is ln((1-p)/p), rounded to
float32 (the decoders consume this float32 value).
"""
from __future__ import annotations

import numpy as np

CHUNK = 8192


def words_for(nbits: int) -> int:
    return (nbits + 63) // 64


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """bool/uint8 [S, n] -> uint64 [S, ceil(n/64)], LSB-first."""
    bits = np.asarray(bits, dtype=np.uint8)
    s, n = bits.shape
    w = words_for(n)
    padded = np.zeros((s, w * 64), dtype=np.uint8)
    padded[:, :n] = bits
    by = np.packbits(padded.reshape(s, w * 8, 8), axis=2, bitorder="little").reshape(s, w * 8)
    return by.view("<u8").reshape(s, w).copy()


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 [S, W] -> uint8 [S, n]."""
    words = np.ascontiguousarray(words, dtype="<u8")
    s, w = words.shape
    by = words.view(np.uint8).reshape(s, w * 8)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :n].copy()


def _threshold(p):
    return np.minimum(np.round(np.asarray(p, dtype=np.float64) * 2.0 ** 32), 2.0 ** 32 - 1).astype(np.uint64)


def bitflip_packed(shots: int, n: int, p, seed: int, stream: int = 0) -> np.ndarray:
    """Packed i.i.d. bit-flip errors [shots, ceil(n/64)].  `p` is a scalar or a
    per-shot array."""
    rng = np.random.default_rng(np.random.PCG64([seed, stream, 0xB17F]))
    p_arr = np.broadcast_to(np.asarray(p, dtype=np.float64), (shots,))
    out = np.empty((shots, words_for(n)), dtype=np.uint64)
    for s0 in range(0, shots, CHUNK):
        s1 = min(shots, s0 + CHUNK)
        u = rng.integers(0, 2 ** 32, size=(s1 - s0, n), dtype=np.uint64)
        thr = _threshold(p_arr[s0:s1])[:, None]
        out[s0:s1] = pack_bits(u < thr)
    return out


def depolarizing_packed(shots: int, n: int, p: float, seed: int, stream: int = 0):
    """Depolarising noise: returns packed (x_part, z_part); a Y error sets
    both.  Each qubit: X, Y, Z with probability p/3 each."""
    rng = np.random.default_rng(np.random.PCG64([seed, stream, 0xDE90]))
    w = words_for(n)
    xs = np.empty((shots, w), dtype=np.uint64)
    zs = np.empty((shots, w), dtype=np.uint64)
    t1, t2, t3 = (_threshold(p / 3.0), _threshold(2 * p / 3.0), _threshold(p))
    for s0 in range(0, shots, CHUNK):
        s1 = min(shots, s0 + CHUNK)
        u = rng.integers(0, 2 ** 32, size=(s1 - s0, n), dtype=np.uint64)
        is_x = u < t1
        is_y = (u >= t1) & (u < t2)
        is_z = (u >= t2) & (u < t3)
        xs[s0:s1] = pack_bits(is_x | is_y)
        zs[s0:s1] = pack_bits(is_z | is_y)
    return xs, zs


def uniform_p(shots: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.PCG64([seed, 0x9A17]))
    return rng.uniform(lo, hi, size=shots)


def channel_llr(p) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    return np.log((1.0 - p) / p).astype(np.float32)
