"""Pins of the Grain oracle (oracle/grain_ref.c) to facts outside itself:

- the known-answer keystreams of the Grain specification (tests/golden), which fix the
  feedback and output functions, the initialisation and every bit-order convention;
- primitivity of the LFSR's feedback polynomial, read off the oracle's clock (a wrong
  or missing tap almost surely breaks it);
- the filter function h's published design properties (balanced, correlation immune of
  order one, algebraic degree 3, nonlinearity 12), computed from its truth table;
- locality: the LFSR feeds the NFSR only through its oldest bit, and keystream
  generation never adds the output bit back into the registers;
- split generation equals one generation, and many instances equal single ones.
"""
import os

import numpy as np
import pytest

from oracle import grain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "grain_v1_kat.txt")


def load_kats():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        f = dict(kv.split("=") for kv in line.split())
        out.append((bytes.fromhex(f["key"]), bytes.fromhex(f["iv"]), bytes.fromhex(f["ks"])))
    return out


def test_known_answer_keystreams():
    kats = load_kats()
    assert len(kats) == 2
    for key, iv, ks in kats:
        assert grain.keystream(key, iv, 8 * len(ks)) == ks


# ---------------------------------------------------------------- LFSR polynomial

def poly_mulmod(a, b, p, deg):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if (a >> deg) & 1:
            a ^= p
    return r


def poly_powmod(e, p, deg):
    r, base = 1, 2
    while e:
        if e & 1:
            r = poly_mulmod(r, base, p, deg)
        base = poly_mulmod(base, base, p, deg)
        e >>= 1
    return r


# 2^80 - 1 = (2^40 - 1)(2^40 + 1) = 3 * 5^2 * 11 * 17 * 31 * 41 * 257 * 61681 * 4278255361
PRIMES_2_80_M1 = [3, 5, 11, 17, 31, 41, 257, 61681, 4278255361]


def test_factorisation_of_group_order():
    n = 1
    for p, e in zip(PRIMES_2_80_M1, [1, 2] + [1] * 7):
        n *= p ** e
    assert n == (1 << 80) - 1
    for p in PRIMES_2_80_M1:  # each factor is prime (trial division)
        assert all(p % d for d in range(2, int(p ** 0.5) + 1)), p


def lfsr_taps():
    """Offsets k with s_{i+80} = sum s_{i+k}: probe the feedback with one bit set."""
    taps = []
    for k in range(80):
        st = grain.State()
        st.s[k] = 1
        if st.lfsr_feedback():
            taps.append(k)
    return taps


def test_lfsr_polynomial_is_primitive():
    taps = lfsr_taps()
    # characteristic polynomial of s_{i+80} = sum_{k in taps} s_{i+k}
    p = (1 << 80) | sum(1 << k for k in taps)
    order = (1 << 80) - 1
    assert poly_powmod(order, p, 80) == 1
    for q in PRIMES_2_80_M1:
        assert poly_powmod(order // q, p, 80) != 1, q


def test_lfsr_feedback_is_linear():
    rng = np.random.default_rng(1)
    for _ in range(50):
        a, b = grain.State(), grain.State()
        a.s[:] = rng.integers(0, 2, 80)
        b.s[:] = rng.integers(0, 2, 80)
        c = grain.State()
        c.s[:] = a.s ^ b.s
        assert c.lfsr_feedback() == a.lfsr_feedback() ^ b.lfsr_feedback()


# ---------------------------------------------------------------- filter function h

def walsh(tt, nvars):
    return [sum((-1) ** (tt[x] ^ (bin(x & w).count("1") & 1)) for x in range(1 << nvars)) for w in range(1 << nvars)]


def anf_degree(tt, nvars):
    a = list(tt)
    for i in range(nvars):  # Moebius transform
        for x in range(1 << nvars):
            if x >> i & 1:
                a[x] ^= a[x ^ (1 << i)]
    return max((bin(x).count("1") for x in range(1 << nvars) if a[x]), default=0)


def test_filter_h_design_properties():
    tt = [grain.h(*[(x >> i) & 1 for i in range(5)]) for x in range(32)]
    w = walsh(tt, 5)
    assert w[0] == 0  # balanced
    assert all(w[1 << i] == 0 for i in range(5))  # correlation immune of order one
    assert anf_degree(tt, 5) == 3
    assert 16 - max(abs(v) for v in w) // 2 == 12  # nonlinearity


# ---------------------------------------------------------------- clock structure

def test_nfsr_takes_lfsr_only_through_oldest_bit():
    rng = np.random.default_rng(2)
    for _ in range(30):
        st = grain.State()
        st.buf[:] = rng.integers(0, 2, 160)
        ref = grain.State()
        ref.buf[:] = st.buf
        ref.s[1:] ^= rng.integers(0, 2, 79).astype(np.uint8)  # change every LFSR bit but s_i
        st.clock(False)
        ref.clock(False)
        assert st.b[79] == ref.b[79]


def test_keystream_clock_shifts_and_does_not_feed_output_back():
    rng = np.random.default_rng(3)
    for _ in range(30):
        st = grain.State()
        st.buf[:] = rng.integers(0, 2, 160)
        before = st.buf.copy()
        f_s, g = st.lfsr_feedback(), st.nfsr_g()
        z = st.output()
        assert st.clock(False) == z
        assert (st.b[:79] == before[1:80]).all() and (st.s[:79] == before[81:160]).all()
        assert st.s[79] == f_s and st.b[79] == g ^ before[80]
        st2 = grain.State()
        st2.buf[:] = before
        st2.clock(True)  # initialisation clock: z added to both feedbacks
        assert st2.s[79] == f_s ^ z and st2.b[79] == g ^ before[80] ^ z


def test_state_pack_roundtrip():
    rng = np.random.default_rng(4)
    st = grain.State()
    st.buf[:] = rng.integers(0, 2, 160)
    p = st.packed()
    other = grain.State()
    other.unpack(p)
    assert (other.buf == st.buf).all()
    assert st.b[0] == p[0] & 1 and st.s[0] == p[10] & 1 and st.b[79] == p[9] >> 7


def test_split_generation_equals_whole():
    key, iv = bytes(range(10)), bytes(range(8))
    st = grain.State()
    st.init(key, iv)
    a = st.generate(96)
    b = st.generate(160)
    whole = np.unpackbits(np.frombuffer(grain.keystream(key, iv, 256), dtype=np.uint8), bitorder="little")
    got = np.concatenate([np.unpackbits(np.frombuffer(x, dtype=np.uint8), bitorder="little") for x in (a, b)])
    assert (got == whole).all()


def test_generate_many_matches_single_and_skip():
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 256, (9, 10), dtype=np.uint8)
    ivs = rng.integers(0, 256, (9, 8), dtype=np.uint8)
    many = grain.generate_many(keys, ivs, 200, threads=3)
    for i in range(9):
        assert many[i].tobytes() == grain.keystream(keys[i].tobytes(), ivs[i].tobytes(), 200)
    skipped = grain.generate_many(keys, ivs, 64, skip=136)
    full = np.unpackbits(many, axis=1, bitorder="little")
    assert (np.unpackbits(skipped, axis=1, bitorder="little") == full[:, 136:200]).all()
