"""CPU checks of the generated MICKEY-128 2.0 loops (paper_1909_04750_amd/csrc/mickey128_loops.inc):

- the committed file is what gen_m128_loop.py produces;
- every register each body reads is a state or import register or was written before;
- run region by region by the register-level emulator of tests/asm_emulator.py, with the
  other wave's side of each exchange taken from the oracle's trajectory, the R body stores
  the oracle's keystream bit of every clock and exports the oracle's r_53, the S body
  exports the oracle's s_54 and s_0, and both end on the oracle's registers (paper Sec.
  IV-D: bitslicing changes only the layout, so each bit of a word is one instance).
"""
import importlib.util
import os
import re

import numpy as np

from oracle import mickey128 as m128
from tests import asm_emulator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "mickey128_loops.inc")
N = 160
LANES, ITERS = 2, 3
# XLds: r53, s54, s0, s80, each [2][64] words
SLOT = {"r53": 0, "s54": 128, "s0": 256}


def generator():
    spec = importlib.util.spec_from_file_location("gen_m128_loop", os.path.join(CSRC, "gen_m128_loop.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def parse(wave):
    text = open(INC).read()
    body = re.search(r"#define M128_%s_LOOP_BODY \\\n(.*?)\n#define" % wave, text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    state = re.search(r"#define M128_%s_LOOP_STATE\([^)]*\) \\\n(.*?)\n#define" % wave, text, re.S).group(1)
    homes = [(int(v), name, int(i) if i else None)
             for v, name, i in re.findall(r'"\+\{v(\d+)\}"\(((?:R|S)\((\d+)\)|S54|S0|R53)\)', state)]
    return insts, homes


def regions(insts):
    out, cur = [], []
    for ins in insts:
        cur.append(ins)
        if ins.startswith("s_barrier"):
            out.append(cur)
            cur = []
    out.append(cur)
    return out


def test_committed_loops_match_generator():
    assert generator().render() == open(INC).read()


def test_registers_written_before_read():
    for wave in ("R", "S"):
        insts, homes = parse(wave)
        assert asm_emulator.written_before_read(insts, [(v, "H", 0) for v, _, _ in homes]), wave


def words(bits):
    """bits[lane][bit] (0/1) -> uint32 array over lanes."""
    return np.array([sum(int(b) << k for k, b in enumerate(lane_bits)) for lane_bits in bits], dtype=np.uint32)


def trajectory(seed):
    """Per clock t: (r words, s words), each a function of the position."""
    rng = np.random.default_rng(seed)
    clocks = 2 * ITERS
    tr = np.zeros((clocks + 1, LANES, 32, N), dtype=np.uint8)
    ts = np.zeros((clocks + 1, LANES, 32, N), dtype=np.uint8)
    for lane in range(LANES):
        for b in range(32):
            st = m128.State()
            st.r[:] = rng.integers(0, 2, N)
            st.s[:] = rng.integers(0, 2, N)
            for t in range(clocks + 1):
                tr[t, lane, b] = st.r
                ts[t, lane, b] = st.s
                st.clock_kg(0, 0)
    return (lambda t, i: words(tr[t, :, :, i])), (lambda t, i: words(ts[t, :, :, i])), rng


def run(wave, seed):
    insts, homes = parse(wave)
    regs_by_region = regions(insts)
    assert len(regs_by_region) == 3  # two barriers per iteration
    word_r, word_s, rng = trajectory(seed)
    regs = {v: rng.integers(0, 2 ** 32, LANES, dtype=np.uint64).astype(np.uint32) for v in range(256)}
    for v, name, i in homes:
        regs[v] = {"R": lambda: word_r(0, i), "S": lambda: word_s(0, i), "S54": lambda: word_s(0, 54),
                   "S0": lambda: word_s(0, 0), "R53": lambda: word_r(0, 53)}[name[0] if name[0] in "RS" and i is not None
                                                                           else name]()
    lds = np.zeros(4 * 2 * 64, dtype=np.uint32)
    addr = {"xaddr": np.arange(LANES) * 4}
    stored = []
    t = 0
    for _ in range(ITERS):
        for k in range(3):
            stored += asm_emulator.emulate(regs_by_region[k], regs, lds, addr)
            if k < 2:  # clock t's barrier: exchange parity (t + 1) & 1
                ph = (t + 1) & 1

                def slot(name):
                    return slice(SLOT[name] + 64 * ph, SLOT[name] + 64 * ph + LANES)
                if wave == "R":
                    assert np.array_equal(lds[slot("r53")], word_r(t + 1, 53)), ("r53", t)
                    lds[slot("s54")] = word_s(t + 1, 54)
                    lds[slot("s0")] = word_s(t + 1, 0)
                else:
                    assert np.array_equal(lds[slot("s54")], word_s(t + 1, 54)), ("s54", t)
                    assert np.array_equal(lds[slot("s0")], word_s(t + 1, 0)), ("s0", t)
                    lds[slot("r53")] = word_r(t + 1, 53)
                t += 1
    clocks = 2 * ITERS
    assert t == clocks
    if wave == "R":
        assert len(stored) == clocks
        for c in range(clocks):
            assert np.array_equal(stored[c], word_r(c, 0) ^ word_s(c, 0)), ("z", c)
    else:
        assert not stored
    for v, name, i in homes:
        if i is not None:
            want = word_r(clocks, i) if name.startswith("R") else word_s(clocks, i)
            assert np.array_equal(regs[v], want), (name, i)


def test_r_loop_equals_oracle_clocks():
    run("R", 128)


def test_s_loop_equals_oracle_clocks():
    run("S", 129)
