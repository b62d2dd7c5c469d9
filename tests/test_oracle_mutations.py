"""The oracle's pins must catch plausible mistakes.  Each case plants one mistake in a
copy of oracle/mickey_ref.c (on the CPU, in a temporary directory), builds it with gcc,
and checks that the known-answer keystreams or the R-register algebra reject it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests.test_oracle_pins import PRIMES_2_100_M1, load_kats, poly_powmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "mickey_ref.c")).read()

# (name, original text, planted text); every original must occur exactly once
MUTATIONS = [
    ("comp0 bit flip", '"-0001100010111101001"', '"-0001100010111101011"'),
    ("comp1 bit flip", '"01101011101111000110"', '"01101011101111000100"'),
    ("fb0 bit flip", '"11001001010100101111"', '"11001001010100101110"'),
    ("fb1 bit flip", '"11011111000000100001"', '"11011111000000100011"'),
    ("rtaps wrong tap", "94, 95, 96, 97};", "94, 95, 96, 98};"),
    ("feedback tables swapped", "(control_bit_s & 1) ? tab(FB1, i) : tab(FB0, i)",
     "(control_bit_s & 1) ? tab(FB0, i) : tab(FB1, i)"),
    ("control bit r index", "st->s[34] ^ st->r[67]", "st->s[35] ^ st->r[67]"),
    ("control bit s index", "st->s[67] ^ st->r[33]", "st->s[67] ^ st->r[32]"),
    ("mixing tap", "((input_bit & 1) ^ st->s[50])", "((input_bit & 1) ^ st->s[51])"),
    ("no mixing", "int input_bit_r = mixing ?", "int input_bit_r = 0 ?"),
    ("s-hat neighbour", "st->s[i - 1] ^ ((st->s[i] ^", "st->s[i + 1] ^ ((st->s[i] ^"),
    ("s-hat last position", "s_hat[99] = st->s[98];", "s_hat[99] = st->s[99];"),
    ("r shift", "r_new[i] = st->r[i - 1];", "r_new[i] = st->r[i];"),
    ("r jump dropped", "r_new[i] ^= st->r[i];", "r_new[i] ^= 0;"),
    ("key bit order LSB first", "return (bytes[j >> 3] >> (7 - (j & 7))) & 1;", "return (bytes[j >> 3] >> (j & 7)) & 1;"),
    ("99 preclocks", "for (unsigned i = 0; i < 100; i++)\n        mref_clock_kg(st, 1, 0);",
     "for (unsigned i = 0; i < 99; i++)\n        mref_clock_kg(st, 1, 0);"),
    ("output uses r0 only", "int z = st->r[0] ^ st->s[0];", "int z = st->r[0];"),
    ("clock before output",
     "int z = st->r[0] ^ st->s[0];\n        out[t >> 3] |= (uint8_t)(z << (7 - (t & 7)));\n        mref_clock_kg(st, 0, 0);",
     "mref_clock_kg(st, 0, 0);\n        int z = st->r[0] ^ st->s[0];\n        out[t >> 3] |= (uint8_t)(z << (7 - (t & 7)));"),
]


def build_variant(tmp_path, name, old, new):
    assert SRC.count(old) == 1, name
    src = tmp_path / "m.c"
    src.write_text(SRC.replace(old, new))
    so = tmp_path / "m.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(src), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.mref_init.argtypes = [ctypes.c_void_p, u8p, u8p, ctypes.c_uint]
    L.mref_generate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p]
    L.mref_clock_r.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    return L


def kats_pass(L):
    for key, iv, L_iv, ks in load_kats():
        st = np.zeros(200, dtype=np.uint8)
        k = np.frombuffer(key, dtype=np.uint8).copy()
        v = np.frombuffer(iv.ljust(10, b"\0"), dtype=np.uint8).copy()
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.mref_init(st.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(u8p), v.ctypes.data_as(u8p), L_iv)
        out = np.zeros(len(ks), dtype=np.uint8)
        L.mref_generate(st.ctypes.data_as(ctypes.c_void_p), 8 * len(ks), out.ctypes.data_as(u8p))
        if out.tobytes() != ks:
            return False
    return True


def r_algebra_pass(L):
    st = np.zeros(200, dtype=np.uint8)
    st[99] = 1
    L.mref_clock_r(st.ctypes.data_as(ctypes.c_void_p), 0, 0)
    p = (1 << 100) | sum(int(b) << i for i, b in enumerate(st[:100]))
    order = (1 << 100) - 1
    if poly_powmod(order, p, 100) != 1 or any(poly_powmod(order // q, p, 100) == 1 for q in PRIMES_2_100_M1):
        return False
    return poly_powmod((1 << 50) - 157, p, 100) == 0b11


def test_unmutated_copy_passes(tmp_path):
    L = build_variant(tmp_path, "none", "mref_state;\n\n/* R feedback", "mref_state;\n\n/* R feedback")
    assert kats_pass(L) and r_algebra_pass(L)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    L = build_variant(tmp_path, name, old, new)
    assert not (kats_pass(L) and r_algebra_pass(L)), name
