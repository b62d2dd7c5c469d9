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
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "mickey_clock_loop.inc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_clock_loop", os.path.join(CSRC, "gen_clock_loop.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def parse_inc():
    text = open(INC).read()
    clocks = int(re.search(r"#define MICKEY_LOOP_CLOCKS (\d+)", text).group(1))
    body = re.search(r"#define MICKEY_LOOP_BODY \\\n(.*?)\n#define", text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    homes = [(int(v), kind, int(idx)) for v, kind, idx in
             re.findall(r'"\+\{v(\d+)\}"\(([RS])\((\d+)\)\)', text)]
    return clocks, insts, homes


def emulate(insts, regs):
    """Run one loop iteration on `regs` (dict vN -> uint32 array); returns stored words."""
    stored = []
    for ins in insts:
        op, _, rest = ins.partition(" ")
        if op in ("s_add_u32", "s_addc_u32"):
            continue
        args = [a.strip() for a in rest.split(",")]
        if op == "buffer_store_dword":
            stored.append(regs[int(args[0][1:])].copy())
            continue
        if op == "v_bitop3_b32":
            d, a, b, c = (int(x.split()[0][1:]) for x in args[:4])
            imm = int(args[3].split("bitop3:")[1], 16)
            va, vb, vc = regs[a], regs[b], regs[c]
            out = np.zeros_like(va)
            for m in range(8):
                if imm >> m & 1:
                    out |= (va if m & 4 else ~va) & (vb if m & 2 else ~vb) & (vc if m & 1 else ~vc)
            regs[d] = out
        elif op in ("v_xor_b32", "v_and_b32"):
            d, a, b = (int(x[1:]) for x in args)
            regs[d] = regs[a] ^ regs[b] if op == "v_xor_b32" else regs[a] & regs[b]
        elif op == "v_mov_b32":
            d, a = (int(x[1:]) for x in args)
            regs[d] = regs[a].copy()
        else:
            raise AssertionError("unexpected instruction " + ins)
    return stored


def test_committed_loop_matches_generator():
    assert generator().render() == open(INC).read()


def test_temporaries_written_before_read():
    _, insts, homes = parse_inc()
    written = {v for v, _, _ in homes}
    for ins in insts:
        op, _, rest = ins.partition(" ")
        if not op.startswith("v_"):
            if op == "buffer_store_dword":
                assert int(rest.split(",")[0].strip()[1:]) in written
            continue
        regs = [int(x.strip().split()[0][1:]) for x in rest.split(",")]
        for src in regs[1:]:
            assert src in written, ins
        written.add(regs[0])


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
