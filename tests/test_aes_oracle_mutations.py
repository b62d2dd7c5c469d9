"""The AES oracle's pins must catch plausible mistakes.  Each case plants one mistake in
a copy of oracle/aes_ref.c (on the CPU, in a temporary directory), builds it with gcc,
and checks that the standards' vectors reject it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from tests.test_aes_oracle_pins import load_kats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "aes_ref.c")).read()

MUTATIONS = [
    ("field polynomial", "if (hi) a ^= 0x1B;", "if (hi) a ^= 0x1D;"),
    ("affine constant", "(0x63 >> i)", "(0x62 >> i)"),
    ("affine rotation", "(b >> ((i + 7) % 8))", "(b >> ((i + 3) % 8))"),
    ("inverse exponent", "for (int i = 0; i < 254; i++)", "for (int i = 0; i < 253; i++)"),
    ("rcon start", "uint8_t rcon = 1;", "uint8_t rcon = 2;"),
    ("no RotWord", "            t[0] = t[1];\n            t[1] = t[2];\n            t[2] = t[3];\n            t[3] = r0;\n",
     "            (void)r0;\n"),
    ("shift rows right", "t[c] = s[r][(c + r) % 4];", "t[c] = s[r][(c + 4 - r) % 4];"),
    ("mix coefficient", "aref_gmul(a[(r + 1) % 4], 3)", "aref_gmul(a[(r + 1) % 4], 2)"),
    ("nine rounds", "for (int round = 1; round < 10; round++)", "for (int round = 1; round < 9; round++)"),
    ("last round mixes", "    sub_bytes(s);\n    shift_rows(s);\n    add_round_key(s, w, 10);",
     "    sub_bytes(s);\n    shift_rows(s);\n    mix_columns(s);\n    add_round_key(s, w, 10);"),
    ("state transposed", "for (int i = 0; i < 16; i++) s[i % 4][i / 4] = in[i];",
     "for (int i = 0; i < 16; i++) s[i / 4][i % 4] = in[i];"),
    ("counter little-endian", "const unsigned add = (i >= 8) ? (unsigned)((j >> (8 * (15 - i))) & 0xFF) : 0u;",
     "const unsigned add = (i < 8) ? (unsigned)((j >> (8 * i)) & 0xFF) : 0u;"),
]


def build_variant(tmp_path, name, old, new):
    assert SRC.count(old) == 1, name
    src = tmp_path / "a.c"
    src.write_text(SRC.replace(old, new))
    so = tmp_path / "a.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(src), "-o", str(so)])
    L = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    L.aref_encrypt.argtypes = [u8p, u8p, u8p]
    L.aref_ctr_many.argtypes = [u8p, u8p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint64, u8p]
    return L


def vectors_pass(L):
    u8p = ctypes.POINTER(ctypes.c_uint8)

    def p(b):
        return np.frombuffer(b, dtype=np.uint8).copy()
    blocks, ctrs = load_kats()
    for f in blocks:
        k, i, o = p(f["key"]), p(f["in"]), np.zeros(16, dtype=np.uint8)
        L.aref_encrypt(k.ctypes.data_as(u8p), i.ctypes.data_as(u8p), o.ctypes.data_as(u8p))
        if o.tobytes() != f["out"]:
            return False
    for f in ctrs:
        k, t, o = p(f["key"]), p(f["t1"]), np.zeros(64, dtype=np.uint8)
        L.aref_ctr_many(k.ctypes.data_as(u8p), t.ctypes.data_as(u8p), 1, 0, 4, o.ctypes.data_as(u8p))
        if o.tobytes() != b"".join(f["o%d" % j] for j in range(1, 5)):
            return False
    return True


def test_unmutated_copy_passes(tmp_path):
    L = build_variant(tmp_path, "none", "uint8_t rcon = 1;", "uint8_t rcon = 1;")
    assert vectors_pass(L)


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(tmp_path, name, old, new):
    assert not vectors_pass(build_variant(tmp_path, name, old, new)), name
