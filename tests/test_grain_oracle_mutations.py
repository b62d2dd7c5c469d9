"""The Grain oracle's pins must catch plausible mistakes.  Each case plants one mistake
in a copy of oracle/grain_ref.c (on the CPU, in a temporary directory), builds it with
gcc, and checks that the known-answer keystreams or the LFSR polynomial reject it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests.test_grain_oracle_pins import PRIMES_2_80_M1, load_kats, poly_powmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "grain_ref.c")).read()

# (name, original text, planted text); every original must occur exactly once
MUTATIONS = [
    ("lfsr wrong tap", "{0, 13, 23, 38, 51, 62}", "{0, 13, 23, 38, 51, 61}"),
    ("output tap", "OUT_TAPS[7] = {1, 2, 4, 10, 31, 43, 56}", "OUT_TAPS[7] = {1, 2, 4, 10, 31, 43, 55}"),
    ("nfsr linear term dropped", "b[14] ^ b[9] ^ b[0]", "b[9] ^ b[0]"),
    ("nfsr quadratic term dropped", "    g ^= b[15] & b[9];\n", ""),
    ("nfsr degree-6 term dropped", "    g ^= b[52] & b[45] & b[37] & b[33] & b[28] & b[21];\n", ""),
    ("nfsr without lfsr bit", "int fb = st->s[0] ^ gref_nfsr_g(st);", "int fb = gref_nfsr_g(st);"),
    ("h inputs swapped", "gref_h(st->s[3], st->s[25], st->s[46]", "gref_h(st->s[3], st->s[46], st->s[25]"),
    ("h term dropped", " ^ (x2 & x3 & x4);", ";"),
    ("159 init clocks", "for (int t = 0; t < 160; t++)", "for (int t = 0; t < 159; t++)"),
    ("init without lfsr feedback", "        fs ^= z;\n", ""),
    ("iv padding zeros", "for (int i = 64; i < 80; i++) st->s[i] = 1;", "for (int i = 64; i < 80; i++) st->s[i] = 0;"),
    ("key bits MSB first", "st->b[i] = (key[i / 8] >> (i % 8)) & 1u;", "st->b[i] = (key[i / 8] >> (7 - i % 8)) & 1u;"),
    ("output bits MSB first", "(uint8_t)(gref_clock(st, 0) << (t % 8))", "(uint8_t)(gref_clock(st, 0) << (7 - t % 8))"),
]


def build_variant(tmp_path, name, old, new):
    assert SRC.count(old) == 1, name
    src = tmp_path / "g.c"
    src.write_text(SRC.replace(old, new))
    so = tmp_path / "g.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(src), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.gref_init.argtypes = [ctypes.c_void_p, u8p, u8p]
    L.gref_generate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, u8p]
    L.gref_lfsr_feedback.argtypes = [ctypes.c_void_p]
    return L


def kats_pass(L):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    for key, iv, ks in load_kats():
        st = np.zeros(160, dtype=np.uint8)
        k = np.frombuffer(key, dtype=np.uint8).copy()
        v = np.frombuffer(iv, dtype=np.uint8).copy()
        L.gref_init(st.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(u8p), v.ctypes.data_as(u8p))
        out = np.zeros(len(ks), dtype=np.uint8)
        L.gref_generate(st.ctypes.data_as(ctypes.c_void_p), 8 * len(ks), out.ctypes.data_as(u8p))
        if out.tobytes() != ks:
            return False
    return True


def lfsr_primitive(L):
    taps = []
    for k in range(80):
        st = np.zeros(160, dtype=np.uint8)
        st[80 + k] = 1
        if L.gref_lfsr_feedback(st.ctypes.data_as(ctypes.c_void_p)):
            taps.append(k)
    p = (1 << 80) | sum(1 << k for k in taps)
    order = (1 << 80) - 1
    return poly_powmod(order, p, 80) == 1 and all(poly_powmod(order // q, p, 80) != 1 for q in PRIMES_2_80_M1)


def test_unmutated_copy_passes(tmp_path):
    L = build_variant(tmp_path, "none", "for (int t = 0; t < 160; t++)", "for (int t = 0; t < 160; t++)")
    assert kats_pass(L) and lfsr_primitive(L)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, name, old, new):
    L = build_variant(tmp_path, name, old, new)
    assert not kats_pass(L), name
    if name == "lfsr wrong tap":
        assert not lfsr_primitive(L)
