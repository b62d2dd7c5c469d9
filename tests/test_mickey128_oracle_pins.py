"""Pins of the MICKEY-128 2.0 oracle (oracle/mickey128_ref.c) against facts fixed outside it.

- R register, probed as a black box through CLOCK_R: the taps read off one clock give a
  primitive degree-160 polynomial P (order of x is 2^160 - 1, all twelve prime factors
  checked), clocking with control bit 1 is multiplication by x + 1 = x^J mod P with
  J = 2^80 - 255, control bit 0 is multiplication by x, and the input bit adds the taps.
- S register: locality of CLOCK_S under single-bit flips, and the four tables read back
  through CLOCK_S probes equal the stand-in recipe (splitmix64, seed 0x128, drawn in the
  order COMP0, COMP1, FB0, FB1, 160 bits each, MSB first, with COMP0/COMP1 unused at 0
  and 159 and FB0_0 = FB1_0 = 1).
- CLOCK_KG: the control bits read s_54/r_106 (for R) and s_106/r_53 (for S), mixing adds
  s_80 to R's input; the keystream bit is r_0 ^ s_0 of the state before the clock.

Parity unpinned here: whether the S tables, the control/mixing positions and the
initialisation order are those of the published MICKEY-128 2.0 (no published vector is
available to this build).
"""
import random

import numpy as np
import pytest
import sympy

from oracle import mickey128 as m128

N = 160
J = (1 << 80) - 255
# 2^160 - 1 = 3 * 5^2 * 11 * 17 * 31 * 41 * 257 * 61681 * 65537 * 414721 * 4278255361 * 44479210368001
FACTORS = {3: 1, 5: 2, 11: 1, 17: 1, 31: 1, 41: 1, 257: 1, 61681: 1, 65537: 1, 414721: 1, 4278255361: 1,
           44479210368001: 1}


def poly_mulmod(a, b, p, deg=N):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= p
    return r


def poly_powmod(e, p, deg=N):
    r, base = 1, 2
    while e:
        if e & 1:
            r = poly_mulmod(r, base, p, deg)
        base = poly_mulmod(base, base, p, deg)
        e >>= 1
    return r


def r_int(st):
    return sum(int(b) << i for i, b in enumerate(st.r))


def set_r(st, v):
    st.r[:] = [(v >> i) & 1 for i in range(N)]


def feedback_poly():
    st = m128.State()
    set_r(st, 1 << (N - 1))
    st.clock_r(0, 0)
    return (1 << N) | r_int(st)


def copy(st):
    c = m128.State()
    c.buf[:] = st.buf
    return c


def random_state(rng):
    st = m128.State()
    st.buf[:] = np.array([rng.getrandbits(1) for _ in range(2 * N)], dtype=np.uint8)
    return st


# ------------------------------------------------------------------------- R register

def test_group_order_factorisation():
    n = 1
    for p, e in FACTORS.items():
        assert sympy.isprime(p), p
        n *= p ** e
    assert n == (1 << N) - 1


def test_r_polynomial_is_primitive():
    p = feedback_poly()
    assert bin(p ^ (1 << N)).count("1") == 78 and p & 1  # 78 taps, tap 0 included
    order = (1 << N) - 1
    assert poly_powmod(order, p) == 1
    for q in FACTORS:
        assert poly_powmod(order // q, p) != 1, q


def test_r_control_one_is_jump_by_J():
    assert poly_powmod(J, feedback_poly()) == 0b11


def test_clock_r_is_multiplication_mod_p():
    p = feedback_poly()
    taps = p ^ (1 << N)
    rng = random.Random(17)
    st = m128.State()
    for _ in range(150):
        v = rng.getrandbits(N)
        for ctl, mult in ((0, 0b10), (1, 0b11)):
            for inp in (0, 1):
                set_r(st, v)
                st.clock_r(inp, ctl)
                assert r_int(st) == poly_mulmod(v, mult, p) ^ (taps if inp else 0)


# ------------------------------------------------------------------------- S register

def splitmix64(seed):
    m = (1 << 64) - 1
    x = seed
    while True:
        x = (x + 0x9E3779B97F4A7C15) & m
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        yield z ^ (z >> 31)


def stand_in_tables():
    g = splitmix64(0x128)

    def draw():
        out = []
        while len(out) < N:
            w = next(g)
            out += [(w >> (63 - k)) & 1 for k in range(64)]
        return out[:N]

    c0, c1, f0, f1 = draw(), draw(), draw(), draw()
    c0[0] = c0[N - 1] = c1[0] = c1[N - 1] = 0
    f0[0] = f1[0] = 1
    return [np.array(t, dtype=np.uint8) for t in (c0, c1, f0, f1)]


def s_after(s_bits, inp, ctl):
    st = m128.State()
    st.s[:] = s_bits
    st.clock_s(inp, ctl)
    return st.s.copy()


def test_s_tables_equal_stand_in_recipe():
    """FB0/FB1 from the input bit on a zero register; COMP0 & COMP1 from the zero register;
    COMP0 (COMP1) from a single set bit at i+1 (at i), read at position i."""
    c0, c1, f0, f1 = stand_in_tables()
    zero = np.zeros(N, dtype=np.uint8)
    base = s_after(zero, 0, 0)
    fb0 = s_after(zero, 1, 0) ^ base
    fb1 = s_after(zero, 1, 1) ^ base
    assert (fb0 == f0).all() and (fb1 == f1).all()
    both = base[1:N - 1]
    assert (both == (c0 & c1)[1:N - 1]).all()
    for i in range(1, N - 1):
        e = zero.copy()
        e[i + 1] = 1
        got = s_after(e, 0, 0)[i]
        if i + 1 == N - 1:  # s_159 set: its feedback enters the FB0 positions
            got ^= f0[i]
        assert got == c0[i] & (1 ^ c1[i]), i
        e = zero.copy()
        e[i] = 1
        got = s_after(e, 0, 0)[i]
        assert got == (1 ^ c0[i]) & c1[i], i


def test_clock_s_locality():
    rng = random.Random(23)
    for _ in range(20):
        base = random_state(rng)
        ctl, inp = rng.getrandbits(1), rng.getrandbits(1)
        ref = copy(base)
        ref.clock_s(inp, ctl)
        for j in range(N - 1):
            t = copy(base)
            t.s[j] ^= 1
            t.clock_s(inp, ctl)
            diff = set(np.nonzero(t.s != ref.s)[0].tolist())
            allowed = {i for i in (j - 1, j, j + 1) if 1 <= i <= N - 2} | ({N - 1} if j == N - 2 else set())
            assert diff <= allowed, (j, diff)
            assert j + 1 in diff


# ------------------------------------------------------------------------- CLOCK_KG

def test_clock_kg_control_bit_r():
    p = feedback_poly()
    rng = random.Random(29)
    for _ in range(20):
        v = rng.getrandbits(N)
        for s54 in (0, 1):
            st = m128.State()
            set_r(st, v)
            st.s[54] = s54
            st.clock_kg(0, 0)
            ctl = ((v >> 106) & 1) ^ s54
            assert r_int(st) == poly_mulmod(v, 0b11 if ctl else 0b10, p)


def test_clock_kg_control_bit_s():
    rng = random.Random(31)
    for _ in range(20):
        s = np.array([rng.getrandbits(1) for _ in range(N)], dtype=np.uint8)
        s[N - 1] = 1  # feedback on: the two controls differ by FB0 vs FB1
        for r53 in (0, 1):
            st = m128.State()
            st.s[:] = s
            st.r[53] = r53
            st.clock_kg(0, 0)
            assert (st.s == s_after(s, 0, int(s[106]) ^ r53)).all()


def test_clock_kg_mixing_adds_s80_to_r_input():
    taps = feedback_poly() ^ (1 << N)
    st = m128.State()
    st.s[80] = 1
    st.clock_kg(1, 0)
    assert r_int(st) == taps
    st = m128.State()
    st.s[80] = 1
    st.clock_kg(0, 0)
    assert r_int(st) == 0


def test_keystream_bit_is_r0_xor_s0_before_the_clock():
    rng = random.Random(37)
    for _ in range(10):
        st = random_state(rng)
        want = []
        probe = copy(st)
        for _ in range(64):
            want.append(int(probe.r[0]) ^ int(probe.s[0]))
            probe.clock_kg(0, 0)
        got = np.unpackbits(np.frombuffer(st.generate(64), dtype=np.uint8))
        assert (got == np.array(want, dtype=np.uint8)).all()
        assert (st.buf == probe.buf).all()


# ------------------------------------------------------------------------- interfaces

def test_iv_length_over_128_rejected():
    with pytest.raises(ValueError):
        m128.State().init(bytes(16), bytes(17), 129)


def test_iv_bits_beyond_length_are_ignored():
    key = bytes(range(16))
    a = m128.keystream(key, bytes([0b10110000]), 4, 96)
    b = m128.keystream(key, bytes([0b10111111]) + bytes(range(15)), 4, 96)
    c = m128.keystream(key, bytes([0b10100000]), 4, 96)
    assert a == b and a != c


def test_split_generation_equals_whole():
    key, iv = bytes(range(16)), bytes(range(100, 116))
    whole = np.unpackbits(np.frombuffer(m128.keystream(key, iv, 77, 900), dtype=np.uint8))[:900]
    st = m128.State()
    st.init(key, iv, 77)
    a = np.unpackbits(np.frombuffer(st.generate(301), dtype=np.uint8))[:301]
    b = np.unpackbits(np.frombuffer(st.generate(599), dtype=np.uint8))[:599]
    assert (np.concatenate([a, b]) == whole).all()


def test_generate_many_matches_single():
    rng = np.random.default_rng(1)
    keys = rng.integers(0, 256, (5, 16), dtype=np.uint8)
    ivs = rng.integers(0, 256, (5, 16), dtype=np.uint8)
    ivb = np.array([0, 1, 127, 128, 64], dtype=np.uint8)
    many = m128.generate_many(keys, ivs, ivb, 200, skip=9, threads=2)
    for i in range(5):
        st = m128.State()
        st.init(keys[i].tobytes(), ivs[i].tobytes(), int(ivb[i]))
        st.generate(9)
        assert many[i].tobytes() == st.generate(200)


def test_pack_state_layout():
    rng = random.Random(41)
    st = random_state(rng)
    bits = np.unpackbits(np.frombuffer(st.packed(), dtype=np.uint8))
    assert (bits[:N] == st.r).all() and (bits[N:] == st.s).all()
