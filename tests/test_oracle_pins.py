"""Pins of the CPU oracle against facts fixed outside the oracle itself.

- Known-answer keystreams of the MICKEY 2.0 specification (tests/golden), covering the
  S-register tables, the control-bit wiring, the key/IV loading and the bit orders.
- R register, probed as a black box through the oracle's CLOCK_R: the feedback taps
  read off one clock must give a primitive degree-100 polynomial P (order of x is
  2^100 - 1), clocking with control bit 1 must equal multiplication by x + 1 modulo P,
  which the specification states equals J = 2^50 - 157 ordinary clocks (x^J = x + 1),
  and control bit 0 must equal multiplication by x.
- Locality of CLOCK_S and the CLOCK_KG control/mixing taps, probed by single-bit flips.
"""
import os
import random

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mickey2_kat.txt")


def load_kats():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        out.append((bytes.fromhex(f["key"]), bytes.fromhex(f["iv"]), int(f["iv_bits"]), bytes.fromhex(f["ks"])))
    return out


@pytest.mark.parametrize("kat", load_kats(), ids=lambda k: "ivbits%d" % k[2])
def test_known_answer_keystreams(kat):
    key, iv, iv_bits, ks = kat
    assert oracle.keystream(key, iv, iv_bits, 8 * len(ks)) == ks


def test_iv_bits_beyond_length_are_ignored():
    key, iv, iv_bits, ks = load_kats()[0]  # 32-bit IV
    junk = iv + bytes([0xA5, 0x5A, 0xFF, 0x00, 0x3C, 0x77])
    assert oracle.keystream(key, junk, iv_bits, 8 * len(ks)) == ks
    # a partial-byte IV length only reads the leading bits of its last byte
    a = oracle.keystream(key, bytes([0b10110000]), 4, 64)
    b = oracle.keystream(key, bytes([0b10111111]), 4, 64)
    c = oracle.keystream(key, bytes([0b10100000]), 4, 64)
    assert a == b and a != c


def test_iv_length_over_80_rejected():
    st = oracle.State()
    with pytest.raises(ValueError):
        st.init(bytes(10), bytes(11), 81)


# ---------------------------------------------------------------- R register (GF(2)[x])

def poly_mulmod(a: int, b: int, p: int, deg: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= p
    return r


def poly_powmod(e: int, p: int, deg: int) -> int:
    r, base = 1, 2  # the polynomial x
    while e:
        if e & 1:
            r = poly_mulmod(r, base, p, deg)
        base = poly_mulmod(base, base, p, deg)
        e >>= 1
    return r


# 2^100 - 1 = 3 * 5^3 * 11 * 31 * 41 * 101 * 251 * 601 * 1801 * 4051 * 8101 * 268501
PRIMES_2_100_M1 = [3, 5, 11, 31, 41, 101, 251, 601, 1801, 4051, 8101, 268501]


def test_factorisation_of_group_order():
    n = 1
    for p, e in zip(PRIMES_2_100_M1, [1, 3] + [1] * 10):
        n *= p ** e
    assert n == (1 << 100) - 1


def r_as_int(st: oracle.State) -> int:
    return sum(int(b) << i for i, b in enumerate(st.r))


def set_r(st: oracle.State, value: int) -> None:
    st.r[:] = [(value >> i) & 1 for i in range(100)]


def feedback_poly() -> int:
    """x^100 + T(x), T read off one CLOCK_R from r = x^99 with control 0 and input 0."""
    st = oracle.State()
    set_r(st, 1 << 99)
    st.clock_r(0, 0)
    return (1 << 100) | r_as_int(st)


def test_r_feedback_polynomial_is_primitive():
    p = feedback_poly()
    assert bin(p & ((1 << 100) - 1)).count("1") == 50  # fifty taps, tap 0 included
    order = (1 << 100) - 1
    assert poly_powmod(order, p, 100) == 1
    for q in PRIMES_2_100_M1:
        assert poly_powmod(order // q, p, 100) != 1, q


def test_r_control_one_is_jump_by_J():
    p = feedback_poly()
    J = (1 << 50) - 157
    assert poly_powmod(J, p, 100) == 0b11  # x^J = x + 1 (mod P)


def test_clock_r_is_multiplication_mod_p():
    p = feedback_poly()
    taps = p ^ (1 << 100)
    rng = random.Random(7)
    st = oracle.State()
    for _ in range(200):
        v = rng.getrandbits(100)
        for ctl, mult in ((0, 0b10), (1, 0b11)):
            for inp in (0, 1):
                set_r(st, v)
                st.clock_r(inp, ctl)
                want = poly_mulmod(v, mult, p, 100) ^ (taps if inp else 0)
                assert r_as_int(st) == want


# ---------------------------------------------------------------- S register / KG probes

def random_state(rng):
    st = oracle.State()
    st.buf[:] = np.array([rng.getrandbits(1) for _ in range(200)], dtype=np.uint8)
    return st


def copy_state(st):
    c = oracle.State()
    c.buf[:] = st.buf
    return c


def test_clock_s_locality():
    """Flipping s_j (j < 99) changes only s-hat positions j-1, j, j+1 within 1..99;
    flipping s_99 changes s_98 (neighbour) and feedback positions only."""
    rng = random.Random(11)
    for _ in range(50):
        base = random_state(rng)
        ctl, inp = rng.getrandbits(1), rng.getrandbits(1)
        ref = copy_state(base)
        ref.clock_s(inp, ctl)
        for j in range(99):
            t = copy_state(base)
            t.s[j] ^= 1
            t.clock_s(inp, ctl)
            diff = set(np.nonzero(t.s != ref.s)[0].tolist())
            allowed = {i for i in (j - 1, j, j + 1) if 1 <= i <= 98} | ({99} if j == 98 else set())
            assert diff <= allowed, (j, diff)
            assert j + 1 in diff  # s_j enters s-hat_{j+1} linearly


def test_clock_s_feedback_sets_differ_with_control():
    """The input bit reaches S only through the feedback sets, which depend on control."""
    st0 = oracle.State()
    a, b = copy_state(st0), copy_state(st0)
    a.clock_s(1, 0)
    b.clock_s(1, 1)
    fb0 = a.s.copy()
    fb1 = b.s.copy()
    z = copy_state(st0)
    z.clock_s(0, 0)
    fb0 ^= z.s
    fb1 ^= z.s
    assert fb0[0] == 1 and fb1[0] == 1  # s'_0 is the feedback bit under either control
    assert (fb0 != fb1).any()


def test_clock_kg_control_taps():
    """CLOCK_KG's control bits read s_34/r_67 (for R) and s_67/r_33 (for S): flipping any
    other single bit of a zero state leaves R's clocking as plain x-multiplication."""
    p = feedback_poly()
    rng = random.Random(3)
    for _ in range(20):
        v = rng.getrandbits(100)
        # R only, S zero: control_r = r_67, so R' = R*(x + r_67)
        st = oracle.State()
        set_r(st, v)
        st.clock_kg(0, 0)
        mult = 0b11 if (v >> 67) & 1 else 0b10
        assert r_as_int(st) == poly_mulmod(v, mult, p, 100)
        # same with s_34 set flips R's control
        st = oracle.State()
        set_r(st, v)
        st.s[34] = 1
        st.clock_kg(0, 0)
        mult = 0b10 if (v >> 67) & 1 else 0b11
        assert r_as_int(st) == poly_mulmod(v, mult, p, 100)


def test_clock_kg_mixing_adds_s50_to_r_input():
    p = feedback_poly()
    taps = p ^ (1 << 100)
    st = oracle.State()
    st.s[50] = 1
    st.clock_kg(1, 0)
    assert r_as_int(st) == taps  # feedback = r_99 ^ (0 ^ s_50) = 1
    st = oracle.State()
    st.s[50] = 1
    st.clock_kg(0, 0)
    assert r_as_int(st) == 0


def test_state_pack_roundtrip():
    rng = random.Random(5)
    st = random_state(rng)
    packed = st.packed()
    bits = np.unpackbits(np.frombuffer(packed, dtype=np.uint8))
    assert (bits[:100] == st.r).all() and (bits[100:] == st.s).all()
    t = oracle.State()
    t.unpack(packed)
    assert (t.buf == st.buf).all()


def test_split_generation_equals_whole():
    key, iv, iv_bits, _ = load_kats()[1]
    whole = oracle.keystream(key, iv, iv_bits, 1000)
    st = oracle.State()
    st.init(key, iv, iv_bits)
    a = np.unpackbits(np.frombuffer(st.generate(333), dtype=np.uint8))[:333]
    b = np.unpackbits(np.frombuffer(st.generate(667), dtype=np.uint8))[:667]
    w = np.unpackbits(np.frombuffer(whole, dtype=np.uint8))[:1000]
    assert (np.concatenate([a, b]) == w).all()


def test_generate_many_matches_single():
    rng = np.random.default_rng(0)
    keys = rng.integers(0, 256, (5, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (5, 10), dtype=np.uint8)
    ivb = np.array([0, 1, 79, 80, 13], dtype=np.uint8)
    many = oracle.generate_many(keys, ivs, ivb, 300, skip=7, threads=2)
    for i in range(5):
        st = oracle.State()
        st.init(keys[i].tobytes(), ivs[i].tobytes(), int(ivb[i]))
        st.generate(7)
        assert many[i].tobytes() == st.generate(300)
