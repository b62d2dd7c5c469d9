"""Pins of the AES oracle (oracle/aes_ref.c) to facts outside itself:

- FIPS-197's cipher example and AES-128 example vector, and the CTR-AES128 vectors of
  NIST SP 800-38A (tests/golden), which fix the S-box, key schedule, round structure,
  byte order and the counter increment;
- FIPS-197's worked S-box example ({53} -> {ed}) and its inverse example ({53}{ca} = {01});
- published properties of the S-box computed from all 256 values: a permutation without
  fixed or complementary fixed points, differential uniformity 4, nonlinearity 112,
  algebraic degree 7;
- MixColumns followed by FIPS-197's InvMixColumns coefficients ({0e},{0b},{0d},{09}) is
  the identity;
- the counter increment is a 128-bit big-endian addition with carry.
"""
import os

import numpy as np

from oracle import aes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "aes128_kat.txt")


def load_kats():
    blocks, ctrs = [], []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, *fields = line.split()
        f = {k: bytes.fromhex(v) for k, v in (x.split("=") for x in fields)}
        (blocks if kind == "block" else ctrs).append(f)
    return blocks, ctrs


def test_block_vectors():
    blocks, _ = load_kats()
    assert len(blocks) == 2
    for f in blocks:
        assert aes.encrypt(f["key"], f["in"]) == f["out"]


def test_ctr_vectors():
    _, ctrs = load_kats()
    (f,) = ctrs
    ks = aes.ctr_many(f["key"], np.frombuffer(f["t1"], dtype=np.uint8).reshape(1, 16), 4)[0].tobytes()
    for j in range(4):
        o = ks[16 * j:16 * j + 16]
        assert o == f["o%d" % (j + 1)]
        assert bytes(a ^ b for a, b in zip(o, f["p%d" % (j + 1)])) == f["c%d" % (j + 1)]
    skipped = aes.ctr_many(f["key"], np.frombuffer(f["t1"], dtype=np.uint8).reshape(1, 16), 2, skip=2)[0]
    assert skipped.tobytes() == ks[32:]


def test_worked_examples():
    assert aes.sbox(0x53) == 0xED
    assert aes.gmul(0x53, 0xCA) == 0x01
    assert aes.gmul(0x57, 0x83) == 0xC1  # FIPS-197 Sec. 4.2
    assert aes.gmul(0x57, 0x13) == 0xFE  # FIPS-197 Sec. 4.2.1


def sbox_table():
    return np.array([aes.sbox(a) for a in range(256)], dtype=np.int64)


def test_sbox_permutation_without_fixed_points():
    s = sbox_table()
    assert sorted(s.tolist()) == list(range(256))
    a = np.arange(256)
    assert not (s == a).any() and not (s == (a ^ 0xFF)).any()


def test_sbox_differential_uniformity_and_nonlinearity():
    s = sbox_table()
    a = np.arange(256)
    ddt_max = max(np.bincount(s ^ s[a ^ d], minlength=256).max() for d in range(1, 256))
    assert ddt_max == 4
    # Walsh spectrum of every non-zero output mask b: nonlinearity = 128 - max|W| / 2
    parity = np.array([bin(x).count("1") & 1 for x in range(256)])
    walsh_max = 0
    for b in range(1, 256):
        fb = parity[s & b]
        for m in range(256):
            w = int(np.sum(1 - 2 * (fb ^ parity[a & m])))
            walsh_max = max(walsh_max, abs(w))
    assert 128 - walsh_max // 2 == 112


def test_sbox_output_bits_have_degree_seven():
    s = sbox_table()
    for bit in range(8):
        f = list((s >> bit) & 1)
        for i in range(8):  # Moebius transform to the algebraic normal form
            for x in range(256):
                if x >> i & 1:
                    f[x] ^= f[x ^ (1 << i)]
        assert max(bin(x).count("1") for x in range(256) if f[x]) == 7


def test_mixcolumns_inverse():
    """The oracle's field multiplication makes the MixColumns polynomial and FIPS-197's
    InvMixColumns polynomial inverses: ({03}x^3 + {01}x^2 + {01}x + {02}) *
    ({0b}x^3 + {0d}x^2 + {09}x + {0e}) = 1 mod x^4 + 1."""
    a = [0x02, 0x01, 0x01, 0x03]  # coefficients of x^0..x^3
    b = [0x0E, 0x09, 0x0D, 0x0B]
    prod = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            prod[(i + j) % 4] ^= aes.gmul(a[i], b[j])
    assert prod == [1, 0, 0, 0]


def test_counter_increment_carries():
    t = bytes.fromhex("000000000000000000000000ffffffff")
    assert aes.counter_add(t, 1) == bytes.fromhex("00000000000000000000000100000000")
    t = bytes.fromhex("ffffffffffffffffffffffffffffffff")
    assert aes.counter_add(t, 2) == bytes.fromhex("00000000000000000000000000000001")
    t = bytes.fromhex("0102030405060708090a0b0c0d0e0f10")
    assert aes.counter_add(t, 0x0100) == bytes.fromhex("0102030405060708090a0b0c0d0e1010")


def test_key_schedule_last_round_key():
    # FIPS-197 Appendix A.1: the expanded key of 2b7e1516... ends with w[43] = b6630ca6
    w = aes.expand_key(bytes.fromhex("2b7e151628aed2a6abf7158809cf4f3c"))
    assert w[-4:] == bytes.fromhex("b6630ca6")
    assert w[16:20] == bytes.fromhex("a0fafe17")  # w[4]
