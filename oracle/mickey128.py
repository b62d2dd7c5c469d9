"""CPU oracle for MICKEY-128 2.0 keystreams (test infrastructure only).

A plain, bit-serial C implementation (``mickey128_ref.c``) of the 128-bit-key member of
the MICKEY 2.0 family that the paper names (Sec. II-C-1): 160-bit R and S registers,
IVs of 0..128 bits.  It is compiled with gcc into ``libmickey128_oracle.so`` and called
through ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; it shares no code with the HIP library.

Pins (``tests/test_mickey128_oracle_pins.py``): the R register read off CLOCK_R is a
primitive degree-160 polynomial whose control-bit-1 clock is x^J with J = 2^80 - 255;
CLOCK_R is multiplication mod P; locality probes of CLOCK_S and CLOCK_KG.  The S tables
are a stand-in (see the C file) and, like the control/mixing positions and the
initialisation order, parity unpinned: no published vector is available to check them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mickey128_ref.c")
_LIB_PATH = os.path.join(_HERE, "libmickey128_oracle.so")
_lock = threading.Lock()
_lib = None

NBITS_REG = 160
STATE_BYTES = 2 * NBITS_REG  # uint8 r[160], s[160]
KEY_BYTES = 16
MAX_IV_BITS = 128


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (building the checker is not using it)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load(path: str):
    """The oracle library at `path` with its ctypes signatures (tests load planted-mistake
    builds through this too)."""
    L = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.m128_clock_r.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.m128_clock_s.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.m128_clock_kg.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.m128_init.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint]
    L.m128_init.restype = ctypes.c_int
    L.m128_generate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p]
    L.m128_generate_many.argtypes = [u8p, u8p, u8p, ctypes.c_size_t, ctypes.c_uint64,
                                     ctypes.c_uint64, u8p]
    L.m128_generate_many.restype = ctypes.c_int
    L.m128_pack_state.argtypes = [ctypes.c_void_p, u8p]
    L.m128_state_size.restype = ctypes.c_size_t
    assert L.m128_state_size() == STATE_BYTES
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = load(_LIB_PATH)
    return _lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class State:
    """One scalar instance: ``r`` and ``s`` are views of the 160 + 160 register bits."""

    def __init__(self):
        self.buf = np.zeros(STATE_BYTES, dtype=np.uint8)

    @property
    def r(self) -> np.ndarray:
        return self.buf[:NBITS_REG]

    @property
    def s(self) -> np.ndarray:
        return self.buf[NBITS_REG:]

    def _p(self):
        return self.buf.ctypes.data_as(ctypes.c_void_p)

    def clock_r(self, input_bit: int, control_bit: int) -> None:
        lib().m128_clock_r(self._p(), int(input_bit), int(control_bit))

    def clock_s(self, input_bit: int, control_bit: int) -> None:
        lib().m128_clock_s(self._p(), int(input_bit), int(control_bit))

    def clock_kg(self, mixing: int, input_bit: int) -> None:
        lib().m128_clock_kg(self._p(), int(mixing), int(input_bit))

    def init(self, key: bytes, iv: bytes, iv_bits: int) -> None:
        k = np.frombuffer(bytes(key).ljust(KEY_BYTES, b"\0"), dtype=np.uint8).copy()
        v = np.frombuffer(bytes(iv).ljust(KEY_BYTES, b"\0"), dtype=np.uint8).copy()
        if lib().m128_init(self._p(), _u8(k), _u8(v), int(iv_bits)) != 0:
            raise ValueError("iv_bits must be <= 128")

    def generate(self, nbits: int) -> bytes:
        out = np.zeros((nbits + 7) // 8, dtype=np.uint8)
        lib().m128_generate(self._p(), int(nbits), _u8(out))
        return out.tobytes()

    def packed(self) -> bytes:
        out = np.zeros(40, dtype=np.uint8)
        lib().m128_pack_state(self._p(), _u8(out))
        return out.tobytes()


def keystream(key: bytes, iv: bytes, iv_bits: int, nbits: int) -> bytes:
    st = State()
    st.init(key, iv, iv_bits)
    return st.generate(nbits)


def generate_many(keys: np.ndarray, ivs: np.ndarray, iv_bits, nbits: int, skip: int = 0,
                  threads: int = 1) -> np.ndarray:
    """Keystreams of many instances: uint8 [n, ceil(nbits/8)], MSB-first bits.

    ``keys``/``ivs`` are uint8 [n, 16]; ``iv_bits`` is uint8 [n] or None (128 for all).
    ``threads`` > 1 splits the instances over Python threads (ctypes releases the GIL).
    """
    keys = np.ascontiguousarray(keys, dtype=np.uint8)
    ivs = np.ascontiguousarray(ivs, dtype=np.uint8)
    n = keys.shape[0]
    assert keys.shape == (n, KEY_BYTES) and ivs.shape == (n, KEY_BYTES)
    ivb = None if iv_bits is None else np.ascontiguousarray(iv_bits, dtype=np.uint8)
    row = (nbits + 7) // 8
    out = np.zeros((n, row), dtype=np.uint8)
    L = lib()
    errs = []

    def run(a: int, b: int) -> None:
        if b <= a:
            return
        rc = L.m128_generate_many(_u8(keys[a:b]), _u8(ivs[a:b]), None if ivb is None else _u8(ivb[a:b]),
                                  b - a, int(skip), int(nbits), _u8(out[a:b]))
        if rc != 0:
            errs.append(ValueError("iv_bits must be <= 128"))

    threads = max(1, min(int(threads), n))
    bounds = [n * k // threads for k in range(threads + 1)]
    ts = [threading.Thread(target=run, args=(bounds[k], bounds[k + 1])) for k in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if errs:
        raise errs[0]
    return out
