"""Test-side layout codec: converts per-instance keystream bit rows (the oracle's
MSB-first packed bytes) to the library's output layouts for comparison.  Pure data
movement; no cipher arithmetic."""
from __future__ import annotations

import numpy as np


def bits_matrix(rows: np.ndarray, nbits: int) -> np.ndarray:
    """uint8 [n, ceil(nbits/8)] MSB-first rows -> uint8 [n, nbits] of 0/1."""
    return np.unpackbits(rows, axis=1)[:, :nbits]


def to_bitsliced(bits: np.ndarray, n_pad: int) -> np.ndarray:
    """[n, nbits] bits -> [nbits, n_pad/8] plane bytes (instance i = bit i%8 of byte i/8)."""
    n, nbits = bits.shape
    planes = np.zeros((nbits, n_pad), dtype=np.uint8)
    planes[:, :n] = bits.T
    return np.packbits(planes, axis=1, bitorder="little")


def from_bitsliced(planes: np.ndarray, n: int) -> np.ndarray:
    """[nbits, pitch] plane bytes -> [n, nbits] bits."""
    return np.unpackbits(planes, axis=1, bitorder="little")[:, :n].T.copy()


def to_rowmajor_u32(bits: np.ndarray) -> np.ndarray:
    """[n, nbits] bits -> uint32 [n, nbits/32]; bit 31-b of word j is bit 32j+b."""
    n, nbits = bits.shape
    assert nbits % 32 == 0
    b = bits.reshape(n, nbits // 32, 32).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(31, -1, -1, dtype=np.uint64))
    return (b * weights).sum(axis=2).astype(np.uint32)


def u32_to_f32(words: np.ndarray) -> np.ndarray:
    """(w >> 8) * 2^-24 in float64 (exact), then cast to float32 (exact: 24-bit values)."""
    return ((words >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
