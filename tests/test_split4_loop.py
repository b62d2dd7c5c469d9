"""CPU checks of the generated four-wave split loop (paper_1909_04750_amd/csrc/mickey_split4_loop.inc):

- the committed file is what gen_split4_loop.py produces;
- the four role bodies, run region by region by the register-level emulator of
  tests/asm_emulator.py with one shared LDS (each s_barrier ends a region for all four waves
  at once), store the keystream of every lane and leave the register halves and the
  exchanged words that the oracle gives for those instances (paper Sec. IV-D);
- every temporary of each role is written before it is read.
"""
import importlib.util
import os
import re

import numpy as np

import oracle
from tests import asm_emulator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "mickey_split4_loop.inc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_split4_loop", os.path.join(CSRC, "gen_split4_loop.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def parse_role(text, role):
    body = re.search(r"#define MICKEY_S4_BODY_%d \\\n(.*?)\n#define" % role, text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    state = re.search(r"#define MICKEY_S4_STATE_%d \\\n(.*?)\n#define" % role, text, re.S).group(1)
    homes = re.findall(r'"\+\{v(\d+)\}"\(([^)]*\)?)\)', state)
    return insts, [(int(v), b) for v, b in homes]


def regions(insts):
    out, cur = [], []
    for ins in insts:
        cur.append(ins)
        if ins.startswith("s_barrier"):
            out.append(cur)
            cur = []
    out.append(cur)
    return out


def test_committed_loop_matches_generator():
    assert generator().render() == open(INC).read()


def test_temporaries_written_before_read():
    text = open(INC).read()
    for role in range(4):
        insts, homes = parse_role(text, role)
        assert asm_emulator.written_before_read(insts, [(v, "H", 0) for v, _ in homes]), role


def test_split4_loop_equals_oracle_clocks():
    text = open(INC).read()
    rng = np.random.default_rng(44)
    lanes, iters = 2, 3
    full_r = rng.integers(0, 2 ** 32, (100, lanes), dtype=np.uint64).astype(np.uint32)
    full_s = rng.integers(0, 2 ** 32, (100, lanes), dtype=np.uint64).astype(np.uint32)
    # what each binding holds at loop entry: a role's half, and the exchanged words of state 0
    imports = {0: {"in.a": full_r[99], "in.b": full_r[67], "in.c": full_s[34], "in.d": full_s[0]},
               1: {"x.r[49]": full_r[49], "in.a": full_s[34]},
               2: {"x.s[50]": full_s[50], "in.a": full_s[99], "in.b": full_s[67], "in.c": full_r[33]},
               3: {"x.s[49]": full_s[49], "in.a": full_r[33]}}
    roles = []
    for role in range(4):
        insts, homes = parse_role(text, role)
        regs = {v: rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for v in range(256)}
        for v, binding in homes:
            # a role's own words and its boundary import are both words of state 0
            m = re.match(r"x\.([rs])\[(\d+)\]\.w\[0\]", binding)
            if m:
                regs[v] = (full_r if m.group(1) == "r" else full_s)[int(m.group(2))].copy()
            else:
                regs[v] = imports[role][binding.replace(".w[0]", "")].copy()
        roles.append((regions(insts), regs, homes))
    lds = np.zeros(2 * 10 * 64, dtype=np.uint32)
    addr = {"xaddr": np.arange(lanes) * 4}
    stored = []
    for _ in range(iters):
        for k in range(3):
            for role, (regs_list, regs, _) in enumerate(roles):
                words = asm_emulator.emulate(regs_list[k], regs, lds, addr)
                if role == 0:
                    stored += words
                else:
                    assert not words
    assert len(stored) == 2 * iters
    for lane in range(lanes):
        for bit in (0, 13, 31):
            st = oracle.State()
            st.r[:] = [(int(full_r[i][lane]) >> bit) & 1 for i in range(100)]
            st.s[:] = [(int(full_s[i][lane]) >> bit) & 1 for i in range(100)]
            want = np.unpackbits(np.frombuffer(st.generate(2 * iters), dtype=np.uint8))[:2 * iters]
            assert [(int(w[lane]) >> bit) & 1 for w in stored] == list(want), (lane, bit)
            for role, (_, regs, homes) in enumerate(roles):
                for v, binding in homes:
                    m = re.match(r"x\.([rs])\[(\d+)\]\.w\[0\]", binding)
                    if not m:
                        continue
                    name, pos = m.group(1), int(m.group(2))
                    arr = st.r if name == "r" else st.s
                    assert (int(regs[v][lane]) >> bit) & 1 == arr[pos], (role, binding, lane, bit)
