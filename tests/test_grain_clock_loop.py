"""CPU checks of the generated Grain keystream loop (paper_1909_04750_amd/csrc/grain_clock_loop.inc):

- the committed file is what gen_grain_loop.py produces;
- its instruction stream, run by the register-level emulator of tests/asm_emulator.py over
  two iterations (160 clocks), gives for every lane of every word the keystream bits and
  the final NFSR/LFSR words that the Grain oracle gives for that instance (paper Sec. IV-D:
  bitslicing changes only the layout), so the rings also return to their slots;
- every temporary is written before it is read.
"""
import importlib.util
import os

import numpy as np

from oracle import grain as grain_oracle
from tests import asm_emulator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "grain_clock_loop.inc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_grain_loop", os.path.join(CSRC, "gen_grain_loop.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_loop_matches_generator():
    assert generator().render() == open(INC).read()


def test_temporaries_written_before_read():
    _, insts, homes = asm_emulator.parse_inc(INC, "GRAIN")
    assert asm_emulator.written_before_read(insts, homes)


def test_loop_body_equals_oracle_clocks():
    clocks, insts, homes = asm_emulator.parse_inc(INC, "GRAIN")
    assert len(homes) == 160
    rng = np.random.default_rng(80)
    lanes, iters = 4, 2
    regs = {v: rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for v in range(256)}
    start = {(k, i): regs[v].copy() for v, k, i in homes}
    stored = []
    for _ in range(iters):
        stored += asm_emulator.emulate(insts, regs)
    assert len(stored) == clocks * iters
    for lane in range(lanes):
        for bit in (0, 22, 31):
            st = grain_oracle.State()
            st.b[:] = [(int(start[("B", i)][lane]) >> bit) & 1 for i in range(80)]
            st.s[:] = [(int(start[("S", i)][lane]) >> bit) & 1 for i in range(80)]
            want = [st.clock(False) for _ in range(clocks * iters)]
            got = [(int(w[lane]) >> bit) & 1 for w in stored]
            assert want == got, (lane, bit)
            assert list(st.b) == [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "B"]
            assert list(st.s) == [(int(regs[v][lane]) >> bit) & 1 for v, k, i in homes if k == "S"]
