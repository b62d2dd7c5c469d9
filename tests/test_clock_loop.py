"""CPU checks of the generated keystream loop (paper_1909_04750_amd/csrc/mickey_clock_loop.inc):

- the committed file is what gen_clock_loop.py produces from mickey_bitslice.h's tables;
- its instruction stream, run by a small register-level emulator of the five gfx950
  instructions it uses, gives for every lane of every word the keystream bits and the
  final registers that the oracle gives for that instance (paper Sec. IV-D: bitslicing
  changes only the layout);
- every temporary is written before it is read, so nothing depends on stale registers;
- the state returns to its home registers at the end of each iteration (the loop closes).
"""
import importlib.util
import os

import numpy as np

import oracle
from tests import asm_emulator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "mickey_clock_loop.inc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_clock_loop", os.path.join(CSRC, "gen_clock_loop.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def parse_inc():
    return asm_emulator.parse_inc(INC, "MICKEY")


emulate = asm_emulator.emulate


def test_committed_loop_matches_generator():
    assert generator().render() == open(INC).read()


def test_temporaries_written_before_read():
    _, insts, homes = parse_inc()
    assert asm_emulator.written_before_read(insts, homes)


def test_loop_body_equals_oracle_clocks():
    clocks, insts, homes = parse_inc()
    rng = np.random.default_rng(2024)
    lanes, iters = 2, 3
    regs = {v: rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for v in range(256)}
    start = {(k, i): regs[v].copy() for v, k, i in homes}
    stored = []
    for _ in range(iters):
        stored += emulate(insts, regs)
    assert len(stored) == clocks * iters
    for lane in range(lanes):
        for bit in (0, 5, 17, 31):
            st = oracle.State()
            st.r[:] = [(int(start[("R", i)][lane]) >> bit) & 1 for i in range(100)]
            st.s[:] = [(int(start[("S", i)][lane]) >> bit) & 1 for i in range(100)]
            want = np.unpackbits(np.frombuffer(st.generate(clocks * iters), dtype=np.uint8))[:clocks * iters]
            got = [(int(w[lane]) >> bit) & 1 for w in stored]
            assert list(want) == got, (lane, bit)
            end_r = [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "R"]
            end_s = [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "S"]
            assert list(st.r) == end_r and list(st.s) == end_s, (lane, bit)


MIX_INC = os.path.join(CSRC, "mickey_mix_loop.inc")


def parse_mix():
    import re
    text = open(MIX_INC).read()
    body = re.search(r"#define MICKEY_MIX_BODY \\\n(.*?)\n#define", text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    ins = [int(v) for v in re.findall(r'"\{v(\d+)\}"\(IN\d\)', text)]
    return insts, ins


def test_committed_mix_loop_matches_generator():
    assert generator().render_mix() == open(MIX_INC).read()


def test_mix_loop_equals_oracle_initialisation_clocks():
    """The initialisation body (CLOCK_KG with mixing on, one input word per clock) against
    the oracle's clock, instance by instance (paper Sec. II-C-1: the key and IV bits enter
    both registers, and s_50 R's feedback)."""
    _, _, homes = parse_inc()
    insts, ins = parse_mix()
    assert len(ins) == 2
    assert asm_emulator.written_before_read(insts, list(homes) + [(v, "I", 0) for v in ins])
    rng = np.random.default_rng(2025)
    lanes, iters = 2, 3
    regs = {v: rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for v in range(256)}
    start = {(k, i): regs[v].copy() for v, k, i in homes}
    inputs = []
    for _ in range(iters):
        words = [rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for _ in range(2)]
        inputs += words
        for v, w in zip(ins, words):
            regs[v] = w.copy()
        assert emulate(insts, regs) == []  # no keystream stores
    for lane in range(lanes):
        for bit in (0, 9, 31):
            st = oracle.State()
            st.r[:] = [(int(start[("R", i)][lane]) >> bit) & 1 for i in range(100)]
            st.s[:] = [(int(start[("S", i)][lane]) >> bit) & 1 for i in range(100)]
            for w in inputs:
                st.clock_kg(1, (int(w[lane]) >> bit) & 1)
            end_r = [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "R"]
            end_s = [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "S"]
            assert list(st.r) == end_r and list(st.s) == end_s, (lane, bit)
