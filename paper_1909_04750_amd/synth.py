"""Seeded synthetic inputs: keys, IVs and IV lengths for the generator instances.

This module holds no cipher arithmetic.  It serves both the HIP path and the oracle
(tests and benchmark feed the same arrays to each).  Every draw comes from splitmix64
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
draw j of seed s is mix64(s + (j+1)*GAMMA) with GAMMA = 0x9E3779B97F4A7C15 and the
published xor-shift-multiply finaliser, so any single draw is an O(1) pure function of
(seed, j) and any instance can be regenerated alone for a sampled check.

The paper draws its per-instance 80-bit IVs from an unspecified non-linear expansion of
a pre-stored random set (Sec. IV-D) and does not say where keys come from; these recipes
stand in for both.

Recipes (instance i of n):
  key  bytes = big-endian bytes of draw 4i (8 bytes) then the top 2 bytes of draw 4i+1
  IV   bytes = big-endian bytes of draw 4i+2 then the top 2 bytes of draw 4i+3
  (128-bit keys and IVs: all 8 bytes of draws 4i, 4i+1 and of 4i+2, 4i+3)
  IV length  (mixed-length workloads only) = {0, 32, 64, 80}[draw (4n + i) >> 62]
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def draws(seed: int, idx) -> np.ndarray:
    """splitmix64 draw(s) number ``idx`` (0-based) of the stream seeded with ``seed``."""
    j = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (j + np.uint64(1)) * GAMMA
    return mix64(x)


def _be_bytes(hi64: np.ndarray, lo64: np.ndarray) -> np.ndarray:
    """[k] uint64 pairs -> [k, 10] bytes: 8 big-endian bytes of hi, top 2 bytes of lo."""
    hi = np.asarray(hi64, dtype=np.uint64).astype(">u8").view(np.uint8).reshape(-1, 8)
    lo = np.asarray(lo64, dtype=np.uint64).astype(">u8").view(np.uint8).reshape(-1, 8)[:, :2]
    return np.ascontiguousarray(np.concatenate([hi, lo], axis=1))


def keys_ivs(seed: int, n: int, idx=None):
    """(keys, ivs) as uint8 [k, 10] for instances ``idx`` (default: all ``n``)."""
    i = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    f = np.uint64(4)
    keys = _be_bytes(draws(seed, f * i), draws(seed, f * i + np.uint64(1)))
    ivs = _be_bytes(draws(seed, f * i + np.uint64(2)), draws(seed, f * i + np.uint64(3)))
    return keys, ivs


def grain_keys_ivs(seed: int, n: int, idx=None):
    """Grain inputs: keys uint8 [k, 10] as keys_ivs, IVs uint8 [k, 8] = draw(4i+2)
    big-endian (the 64-bit IV)."""
    i = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    keys, _ = keys_ivs(seed, n, idx)
    x = draws(seed, np.uint64(4) * i + np.uint64(2))
    ivs = x.astype(">u8").view(np.uint8).reshape(-1, 8).copy()
    return keys, ivs


def aes_inputs(seed: int, n: int, idx=None):
    """AES-CTR inputs: the 16-byte key = draws 4n and 4n+1 big-endian (uint8 [16]), and
    nonce i = draw 4i big-endian (uint8 [k, 8])."""
    i = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    kd = draws(seed, np.array([4 * n, 4 * n + 1], dtype=np.uint64))
    key = kd.astype(">u8").view(np.uint8).reshape(16).copy()
    nonces = draws(seed, np.uint64(4) * i).astype(">u8").view(np.uint8).reshape(-1, 8).copy()
    return key, nonces


def keys_ivs128(seed: int, n: int, idx=None):
    """MICKEY-128 inputs: keys and IVs uint8 [k, 16], key i = draws 4i and 4i+1
    big-endian, IV i = draws 4i+2 and 4i+3 big-endian (128 bits each)."""
    i = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    f = np.uint64(4)
    d = [draws(seed, f * i + np.uint64(k)).astype(">u8").view(np.uint8).reshape(-1, 8) for k in range(4)]
    keys = np.ascontiguousarray(np.concatenate(d[:2], axis=1))
    ivs = np.ascontiguousarray(np.concatenate(d[2:], axis=1))
    return keys, ivs


def iv_lengths_mixed(seed: int, n: int, idx=None) -> np.ndarray:
    """IV lengths uniform in {0, 32, 64, 80} bits (uint8 [k])."""
    i = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    sel = (draws(seed, np.uint64(4 * n) + i) >> np.uint64(62)).astype(np.int64)
    return np.array([0, 32, 64, 80], dtype=np.uint8)[sel]


def batch_requests(seed: int, n: int, max_log2: float = 24.0, min_log2: float = 8.0):
    """Fresh requests for the batched workload: (keys, ivs, iv_bits, nbits).

    keys/ivs as keys_ivs(seed, n); IV length of request i = ((draw(4n+i) >> 32) * 81) >> 32
    (uniform in 0..80); keystream length = 32 * floor(2^(min + (max-min)*u) / 32) with
    u = (draw(5n+i) >> 11) * 2^-53, i.e. log-uniform between 2^min and 2^max bits,
    rounded down to whole 32-bit words.  The float power is evaluated here only, and
    both the GPU run and the oracle consume the resulting integer lengths.
    """
    keys, ivs = keys_ivs(seed, n)
    i = np.arange(n, dtype=np.uint64)
    x = draws(seed, np.uint64(4 * n) + i)
    with np.errstate(over="ignore"):
        ivb = (((x >> np.uint64(32)) * np.uint64(81)) >> np.uint64(32)).astype(np.uint8)
    u = (draws(seed, np.uint64(5 * n) + i) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    nbits = (32 * np.floor(2.0 ** (min_log2 + (max_log2 - min_log2) * u) / 32)).astype(np.uint64)
    return keys, ivs, ivb, nbits


def serve_requests(seed: int, nstates: int, rate: float, duration: float, min_bytes: int = 4096,
                   max_bytes: int = 64 << 20):
    """Poisson arrivals for the served workload: (arrival_s, state_ids, nbits).

    Inter-arrival gaps -ln(1-u)/rate with u = (draw(3k) >> 11) * 2^-53; state id of
    arrival k = draw(3k+1) mod nstates (uniform); size = 4 * floor(2^(log2 min + (log2 max
    - log2 min) * u') / 4) bytes with u' from draw(3k+2), i.e. log-uniform between
    min_bytes and max_bytes, in whole 4-byte words; nbits = 8 * size.  Arrivals are
    generated until `duration` seconds.  Draws use stream `seed`.
    """
    n_est = int(rate * duration * 1.2 + 64)
    k = np.arange(3 * n_est, dtype=np.uint64)
    d = draws(seed, k).reshape(n_est, 3)
    u = (d[:, 0] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    t = np.cumsum(-np.log1p(-u) / rate)
    n = int(np.searchsorted(t, duration))
    t = t[:n]
    sid = (d[:n, 1] % np.uint64(nstates)).astype(np.uint32)
    u2 = (d[:n, 2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    lo, hi = np.log2(min_bytes), np.log2(max_bytes)
    size = 4 * np.floor(2.0 ** (lo + (hi - lo) * u2) / 4)
    return t, sid, (8 * size).astype(np.uint64)


def workload(name: str):
    """Named workloads: (seed, n instances, keystream bits per instance, IV-length recipe)."""
    table = {
        # 1024 instances (32 slices x 32 lanes), 80-bit IVs, 4096 bits each
        "plain-1k": (1, 1024, 4096, "80"),
        # 2^22 instances, 80-bit IVs, 8192 bits each (4 GiB of bitsliced output)
        "plain-4m": (2, 1 << 22, 8192, "80"),
        # 2^20 instances, IV lengths in {0,32,64,80}, 65536 bits each, row-major u32+f32
        "rowmajor-1m": (3, 1 << 20, 65536, "mixed"),
        # 10,000 fresh requests, IV lengths 0..80, lengths log-uniform in [2^8, 2^24) bits
        "batch-10k": (4, 10000, None, "batch"),
        # Grain: 2^22 instances, 80-bit keys, 64-bit IVs, 8192 bits each, bitsliced
        "grain-4m": (6, 1 << 22, 8192, "grain"),
        # AES-128-CTR: one key, 2^22 streams with 64-bit nonces, 8192 bits (64 blocks) each
        "aes-4m": (7, 1 << 22, 8192, "aes"),
        # MICKEY-128 2.0: 3 * 2^20 instances (three waves per SIMD), 128-bit keys and IVs,
        # 8192 bits each (3 GiB of bitsliced output)
        "mickey128-3m": (8, 3 << 20, 8192, "128"),
    }
    return table[name]


def workload_inputs(name: str, idx=None):
    """(keys, ivs, iv_bits or None) for a named workload (optionally a subset ``idx``)."""
    seed, n, _, ivr = workload(name)
    keys, ivs = keys_ivs(seed, n, idx)
    ivb = None if ivr == "80" else iv_lengths_mixed(seed, n, idx)
    return keys, ivs, ivb
