"""The MICKEY-128 2.0 oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of oracle/mickey128_ref.c (on the CPU, in a temporary directory),
builds it with gcc, swaps it in for the oracle library and runs the pins; at least one
must fail."""
import os
import subprocess

import pytest

from oracle import mickey128 as m128
from tests import test_mickey128_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "mickey128_ref.c")).read()

PINS = [pins.test_r_polynomial_is_primitive, pins.test_r_control_one_is_jump_by_J,
        pins.test_clock_r_is_multiplication_mod_p, pins.test_s_tables_equal_stand_in_recipe,
        pins.test_clock_s_locality, pins.test_clock_kg_control_bit_r, pins.test_clock_kg_control_bit_s,
        pins.test_clock_kg_mixing_adds_s80_to_r_input, pins.test_keystream_bit_is_r0_xor_s0_before_the_clock,
        pins.test_iv_bits_beyond_length_are_ignored, pins.test_iv_length_over_128_rejected]

# (name, original text, planted text); every original occurs exactly once
MUTATIONS = [
    ("wrong tap", "152, 153, 154, 156, 157};", "152, 153, 154, 156, 158};"),
    ("dropped tap", "     0,   4,   5,   8,", "     0,   4,   4,   8,"),
    ("comp0 bit flip", '"-1010111011110000100"', '"-1010111011110000110"'),
    ("comp1 bit flip", '"1010100100101001011-"', '"1010100100101001001-"'),
    ("fb0 bit flip", '"00000101001001111011"', '"00000101001001111010"'),
    ("fb1 bit flip", '"00110000111111100110"', '"00110000111111101110"'),
    ("feedback tables swapped", "(control_bit_s & 1) ? tab(FB1, i) : tab(FB0, i)",
     "(control_bit_s & 1) ? tab(FB0, i) : tab(FB1, i)"),
    ("complements swapped", "((st->s[i] ^ tab(COMP0, i)) & (st->s[i + 1] ^ tab(COMP1, i)))",
     "((st->s[i] ^ tab(COMP1, i)) & (st->s[i + 1] ^ tab(COMP0, i)))"),
    ("control bit r index", "st->s[54] ^ st->r[106]", "st->s[54] ^ st->r[105]"),
    ("control bit r s-index", "st->s[54] ^ st->r[106]", "st->s[53] ^ st->r[106]"),
    ("control bit s index", "st->s[106] ^ st->r[53]", "st->s[106] ^ st->r[54]"),
    ("mixing tap", "((input_bit & 1) ^ st->s[80])", "((input_bit & 1) ^ st->s[79])"),
    ("no mixing", "int input_bit_r = mixing ?", "int input_bit_r = 0 ?"),
    ("s-hat neighbour", "st->s[i - 1] ^ ((st->s[i] ^", "st->s[i + 1] ^ ((st->s[i] ^"),
    ("s-hat last position", "s_hat[M128_N - 1] = st->s[M128_N - 2];", "s_hat[M128_N - 1] = st->s[M128_N - 1];"),
    ("r shift", "r_new[i] = st->r[i - 1];", "r_new[i] = st->r[i];"),
    ("r jump dropped", "r_new[i] ^= st->r[i];", "r_new[i] ^= 0;"),
    ("r feedback from r_158", "int feedback_bit = st->r[M128_N - 1]", "int feedback_bit = st->r[M128_N - 2]"),
    ("iv bit order LSB first", "return (bytes[j >> 3] >> (7 - (j & 7))) & 1;", "return (bytes[j >> 3] >> (j & 7)) & 1;"),
    ("iv length check", "if (iv_bits > 128)", "if (iv_bits > 129)"),
    ("output uses r0 only", "int z = st->r[0] ^ st->s[0];", "int z = st->r[0];"),
    ("clock before output",
     "int z = st->r[0] ^ st->s[0];\n        out[t >> 3] |= (uint8_t)(z << (7 - (t & 7)));\n        m128_clock_kg(st, 0, 0);",
     "m128_clock_kg(st, 0, 0);\n        int z = st->r[0] ^ st->s[0];\n        out[t >> 3] |= (uint8_t)(z << (7 - (t & 7)));"),
]


def pins_pass() -> bool:
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, pytest.fail.Exception):
            return False
    return True


def test_pins_pass_on_the_oracle():
    assert pins_pass()


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, monkeypatch, name, old, new):
    assert SRC.count(old) == 1, name
    src = tmp_path / "m.c"
    src.write_text(SRC.replace(old, new))
    so = tmp_path / "m.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(src), "-o", str(so)])
    monkeypatch.setattr(m128, "_lib", m128.load(str(so)))
    assert not pins_pass(), name
