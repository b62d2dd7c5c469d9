"""CPU oracle for Grain (version 1) keystreams (test infrastructure only).

A plain, bit-serial C implementation (``grain_ref.c``) of the second stream cipher the
paper bitslices (Sec. II-C, the Grain subsection: two 80-bit shift registers, an 80-bit
key and a 64-bit IV, 160 initialisation clocks), compiled with gcc into
``libgrain_oracle.so`` and called through ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
It shares no code with the HIP library.

Parity-pinned in ``tests/test_grain_oracle_pins.py``: the specification's two
known-answer keystreams, primitivity of the LFSR polynomial and locality probes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grain_ref.c")
_LIB_PATH = os.path.join(_HERE, "libgrain_oracle.so")
_lock = threading.Lock()
_lib = None

STATE_BYTES = 160  # uint8 b[80], s[80]


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
            u8p = ctypes.POINTER(ctypes.c_uint8)
            vp = ctypes.c_void_p
            for f in ("gref_lfsr_feedback", "gref_nfsr_g", "gref_output"):
                getattr(L, f).argtypes = [vp]
                getattr(L, f).restype = ctypes.c_int
            L.gref_h.argtypes = [ctypes.c_int] * 5
            L.gref_h.restype = ctypes.c_int
            L.gref_clock.argtypes = [vp, ctypes.c_int]
            L.gref_clock.restype = ctypes.c_int
            L.gref_init.argtypes = [vp, u8p, u8p]
            L.gref_generate.argtypes = [vp, ctypes.c_uint64, u8p]
            L.gref_generate_many.argtypes = [u8p, u8p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint64, u8p]
            L.gref_pack_state.argtypes = [vp, u8p]
            L.gref_unpack_state.argtypes = [vp, u8p]
            L.gref_state_size.restype = ctypes.c_size_t
            assert L.gref_state_size() == STATE_BYTES
            _lib = L
    return _lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class State:
    """One scalar Grain instance: ``b`` (NFSR) and ``s`` (LFSR) are views of the
    80 + 80 bits, index 0 the oldest."""

    def __init__(self):
        self.buf = np.zeros(STATE_BYTES, dtype=np.uint8)

    @property
    def b(self) -> np.ndarray:
        return self.buf[:80]

    @property
    def s(self) -> np.ndarray:
        return self.buf[80:]

    def _p(self):
        return self.buf.ctypes.data_as(ctypes.c_void_p)

    def lfsr_feedback(self) -> int:
        return lib().gref_lfsr_feedback(self._p())

    def nfsr_g(self) -> int:
        return lib().gref_nfsr_g(self._p())

    def output(self) -> int:
        return lib().gref_output(self._p())

    def clock(self, init: bool) -> int:
        return lib().gref_clock(self._p(), int(bool(init)))

    def init(self, key: bytes, iv: bytes) -> None:
        k = np.frombuffer(bytes(key), dtype=np.uint8).copy()
        v = np.frombuffer(bytes(iv), dtype=np.uint8).copy()
        assert k.size == 10 and v.size == 8
        lib().gref_init(self._p(), _u8(k), _u8(v))

    def generate(self, nbits: int) -> bytes:
        out = np.zeros((nbits + 7) // 8, dtype=np.uint8)
        lib().gref_generate(self._p(), int(nbits), _u8(out))
        return out.tobytes()

    def packed(self) -> bytes:
        out = np.zeros(20, dtype=np.uint8)
        lib().gref_pack_state(self._p(), _u8(out))
        return out.tobytes()

    def unpack(self, packed20: bytes) -> None:
        a = np.frombuffer(packed20, dtype=np.uint8).copy()
        lib().gref_unpack_state(self._p(), _u8(a))


def h(x0: int, x1: int, x2: int, x3: int, x4: int) -> int:
    return lib().gref_h(x0, x1, x2, x3, x4)


def keystream(key: bytes, iv: bytes, nbits: int) -> bytes:
    st = State()
    st.init(key, iv)
    return st.generate(nbits)


def generate_many(keys: np.ndarray, ivs: np.ndarray, nbits: int, skip: int = 0, threads: int = 1) -> np.ndarray:
    """Keystreams of many instances: uint8 [n, ceil(nbits/8)], least significant bit
    first.  ``keys`` uint8 [n, 10], ``ivs`` uint8 [n, 8]; ``threads`` > 1 splits the
    instances over Python threads (ctypes releases the GIL)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint8)
    ivs = np.ascontiguousarray(ivs, dtype=np.uint8)
    n = keys.shape[0]
    assert keys.shape == (n, 10) and ivs.shape == (n, 8)
    row = (nbits + 7) // 8
    out = np.zeros((n, row), dtype=np.uint8)
    L = lib()

    def run(a: int, b: int) -> None:
        if b > a:
            L.gref_generate_many(_u8(keys[a:b]), _u8(ivs[a:b]), b - a, int(skip), int(nbits), _u8(out[a:b]))

    threads = max(1, min(int(threads), n))
    if threads == 1:
        run(0, n)
    else:
        bounds = [n * k // threads for k in range(threads + 1)]
        ts = [threading.Thread(target=run, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    return out
