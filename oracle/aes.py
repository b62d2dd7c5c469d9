"""CPU oracle for AES-128 and its counter-mode keystream (test infrastructure only).

A plain, byte-oriented C implementation (``aes_ref.c``) of the third generator the paper
bitslices (Sec. II-C, AES subsection: AES in counter mode with the S-box as a bit-level
circuit), following FIPS-197 and the counter mode of NIST SP 800-38A, compiled with gcc
into ``libaes_oracle.so`` and called through ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
It shares no code with the HIP library.

Parity-pinned in ``tests/test_aes_oracle_pins.py``: the standards' example vectors and
published properties of the S-box and MixColumns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aes_ref.c")
_LIB_PATH = os.path.join(_HERE, "libaes_oracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (building the checker is not using it)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            u8, u8p, vp = ctypes.c_uint8, ctypes.POINTER(ctypes.c_uint8), ctypes.c_void_p
            L.aref_gmul.argtypes = [u8, u8]
            L.aref_gmul.restype = u8
            L.aref_ginv.argtypes = [u8]
            L.aref_ginv.restype = u8
            L.aref_sbox.argtypes = [u8]
            L.aref_sbox.restype = u8
            L.aref_expand_key.argtypes = [u8p, vp]
            L.aref_encrypt.argtypes = [u8p, u8p, u8p]
            L.aref_counter_add.argtypes = [u8p, ctypes.c_uint64, u8p]
            L.aref_ctr_many.argtypes = [u8p, u8p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint64, u8p]
            _lib = L
    return _lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _arr(b: bytes, n: int) -> np.ndarray:
    a = np.frombuffer(bytes(b), dtype=np.uint8).copy()
    assert a.size == n
    return a


def gmul(a: int, b: int) -> int:
    return int(lib().aref_gmul(a, b))


def ginv(a: int) -> int:
    return int(lib().aref_ginv(a))


def sbox(a: int) -> int:
    return int(lib().aref_sbox(a))


def expand_key(key: bytes) -> bytes:
    w = np.zeros(176, dtype=np.uint8)
    lib().aref_expand_key(_u8(_arr(key, 16)), w.ctypes.data_as(ctypes.c_void_p))
    return w.tobytes()


def encrypt(key: bytes, block: bytes) -> bytes:
    out = np.zeros(16, dtype=np.uint8)
    lib().aref_encrypt(_u8(_arr(key, 16)), _u8(_arr(block, 16)), _u8(out))
    return out.tobytes()


def counter_add(block: bytes, j: int) -> bytes:
    out = np.zeros(16, dtype=np.uint8)
    lib().aref_counter_add(_u8(_arr(block, 16)), int(j), _u8(out))
    return out.tobytes()


def ctr_many(key: bytes, ctr0: np.ndarray, nblocks: int, skip: int = 0, threads: int = 1) -> np.ndarray:
    """CTR keystreams of n streams under one key: uint8 [n, 16 * nblocks]; stream i
    starts at counter block ctr0[i] + skip."""
    ctr0 = np.ascontiguousarray(ctr0, dtype=np.uint8)
    n = ctr0.shape[0]
    assert ctr0.shape == (n, 16)
    k = _arr(key, 16)
    out = np.zeros((n, 16 * nblocks), dtype=np.uint8)
    L = lib()

    def run(a: int, b: int) -> None:
        if b > a:
            L.aref_ctr_many(_u8(k), _u8(ctr0[a:b]), b - a, int(skip), int(nblocks), _u8(out[a:b]))

    threads = max(1, min(int(threads), n))
    if threads == 1:
        run(0, n)
    else:
        bounds = [n * t // threads for t in range(threads + 1)]
        ts = [threading.Thread(target=run, args=(bounds[t], bounds[t + 1])) for t in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    return out
