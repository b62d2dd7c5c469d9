"""CPU oracle for MICKEY 2.0 keystreams (test infrastructure only).

The oracle is a plain, bit-serial C implementation of the cipher the paper accelerates
(Sec. II-C-1 names MICKEY 2.0; Sec. IV-D bitslices 32 instances per word without
changing any instance's output), compiled with gcc into ``libmickey_oracle.so`` and
called through ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with
the HIP library.

Parity-pinned in ``tests/test_oracle_pins.py``: the specification's known-answer
keystreams, the R-register polynomial properties and locality probes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mickey_ref.c")
_LIB_PATH = os.path.join(_HERE, "libmickey_oracle.so")
_lock = threading.Lock()
_lib = None

STATE_BYTES = 200  # uint8 r[100], s[100]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (the checker is built here; building is not using it)."""
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
            L.mref_clock_r.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
            L.mref_clock_s.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
            L.mref_clock_kg.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
            L.mref_init.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint]
            L.mref_init.restype = ctypes.c_int
            L.mref_generate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p]
            L.mref_generate_many.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_uint64,
                                             ctypes.c_uint64, u8p]
            L.mref_generate_many.restype = ctypes.c_int
            L.mref_pack_state.argtypes = [ctypes.c_void_p, u8p]
            L.mref_unpack_state.argtypes = [ctypes.c_void_p, u8p]
            L.mref_state_size.restype = ctypes.c_size_t
            assert L.mref_state_size() == STATE_BYTES
            _lib = L
    return _lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class State:
    """One scalar MICKEY 2.0 instance: ``r`` and ``s`` are views of the 100+100 bits."""

    def __init__(self):
        self.buf = np.zeros(STATE_BYTES, dtype=np.uint8)

    @property
    def r(self) -> np.ndarray:
        return self.buf[:100]

    @property
    def s(self) -> np.ndarray:
        return self.buf[100:]

    def _p(self):
        return self.buf.ctypes.data_as(ctypes.c_void_p)

    def clock_r(self, input_bit: int, control_bit: int) -> None:
        lib().mref_clock_r(self._p(), int(input_bit), int(control_bit))

    def clock_s(self, input_bit: int, control_bit: int) -> None:
        lib().mref_clock_s(self._p(), int(input_bit), int(control_bit))

    def clock_kg(self, mixing: int, input_bit: int) -> None:
        lib().mref_clock_kg(self._p(), int(mixing), int(input_bit))

    def init(self, key: bytes, iv: bytes, iv_bits: int) -> None:
        k = np.frombuffer(bytes(key).ljust(10, b"\0"), dtype=np.uint8).copy()
        v = np.frombuffer(bytes(iv).ljust(10, b"\0"), dtype=np.uint8).copy()
        if lib().mref_init(self._p(), _u8(k), _u8(v), int(iv_bits)) != 0:
            raise ValueError("iv_bits must be <= 80")

    def generate(self, nbits: int) -> bytes:
        out = np.zeros((nbits + 7) // 8, dtype=np.uint8)
        lib().mref_generate(self._p(), int(nbits), _u8(out))
        return out.tobytes()

    def packed(self) -> bytes:
        out = np.zeros(25, dtype=np.uint8)
        lib().mref_pack_state(self._p(), _u8(out))
        return out.tobytes()

    def unpack(self, packed25: bytes) -> None:
        a = np.frombuffer(packed25, dtype=np.uint8).copy()
        lib().mref_unpack_state(self._p(), _u8(a))


def keystream(key: bytes, iv: bytes, iv_bits: int, nbits: int) -> bytes:
    st = State()
    st.init(key, iv, iv_bits)
    return st.generate(nbits)


def generate_many(keys: np.ndarray, ivs: np.ndarray, iv_bits, nbits: int, skip: int = 0,
                  threads: int = 1) -> np.ndarray:
    """Keystreams of many instances: returns uint8 [n, ceil(nbits/8)], MSB-first bits.

    ``keys``/``ivs`` are uint8 [n, 10]; ``iv_bits`` is uint8 [n] or None (80 for all).
    ``threads`` > 1 splits the instances over Python threads (ctypes releases the GIL).
    """
    keys = np.ascontiguousarray(keys, dtype=np.uint8)
    ivs = np.ascontiguousarray(ivs, dtype=np.uint8)
    n = keys.shape[0]
    assert keys.shape == (n, 10) and ivs.shape == (n, 10)
    ivb = None if iv_bits is None else np.ascontiguousarray(iv_bits, dtype=np.uint8)
    row = (nbits + 7) // 8
    out = np.zeros((n, row), dtype=np.uint8)
    L = lib()

    def run(a: int, b: int) -> None:
        if b <= a:
            return
        rc = L.mref_generate_many(_u8(keys[a:b]), _u8(ivs[a:b]),
                                  None if ivb is None else _u8(ivb[a:b]),
                                  b - a, int(skip), int(nbits), _u8(out[a:b]))
        if rc != 0:
            raise ValueError("iv_bits must be <= 80")

    threads = max(1, min(int(threads), n))
    if threads == 1:
        run(0, n)
    else:
        bounds = [n * k // threads for k in range(threads + 1)]
        errs = []

        def worker(a, b):
            try:
                run(a, b)
            except Exception as e:  # pragma: no cover - re-raised below
                errs.append(e)

        ts = [threading.Thread(target=worker, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        if errs:
            raise errs[0]
    return out
