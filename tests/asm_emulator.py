"""Register-level emulator of the few gfx950 instructions the generated clock loops use
(v_bitop3_b32, v_xor_b32, v_and_b32, v_mov_b32, buffer_store_dword and the scalar address
updates), for CPU tests of the loops in paper_1909_04750_amd/csrc/*_clock_loop.inc."""
import re

import numpy as np


def parse_inc(path, prefix):
    """(clocks, instructions, homes) of a generated loop file; homes are (vgpr, kind, index)
    from its state operand list."""
    text = open(path).read()
    clocks = int(re.search(r"#define %s_LOOP_CLOCKS (\d+)" % prefix, text).group(1))
    body = re.search(r"#define %s_LOOP_BODY \\\n(.*?)\n#define" % prefix, text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    homes = [(int(v), kind, int(idx)) for v, kind, idx in re.findall(r'"\+\{v(\d+)\}"\(([A-Z])\((\d+)\)\)', text)]
    return clocks, insts, homes


def emulate(insts, regs, lds=None, addr=None):
    """Run the instructions once on `regs` (dict vN -> uint32 array over lanes); returns the
    keystream words in clock order, each an array over lanes.

    LDS and the 16-byte stores follow the generated loops' quad regrouping: lane l writes
    its clock word at byte l*4 + 256*(clock % 4) (%[zaddr] = 4*l), reads 16 bytes at
    ((l % 4)*64 + l - l % 4)*4 (%[qaddr]), and a buffer_store_dwordx4 by lane l holds clock
    (4*group + l % 4)'s words of the lanes of its quad.  The lane count must be a multiple
    of 4 when the loop uses these instructions."""
    lanes = len(next(iter(regs.values())))
    if lds is None:
        lds = np.zeros(4 * 64, dtype=np.uint32)
    if addr is None:  # the quad regrouping's LDS addresses
        addr = {"zaddr": np.arange(lanes) * 4,
                "qaddr": np.array([((l % 4) * 64 + l - l % 4) * 4 for l in range(lanes)])}
    stored = []

    def lds_index(arg, lane):
        name = re.search(r"%\[(\w+)\]", arg).group(1)
        off = int(arg.split("offset:")[1]) if "offset:" in arg else 0
        return (int(addr[name][lane]) + off) // 4
    for ins in insts:
        op, _, rest = ins.partition(" ")
        if op in ("s_add_u32", "s_addc_u32", "s_waitcnt", "s_barrier"):
            continue
        args = [a.strip() for a in rest.split(",")]
        if op == "buffer_store_dword":
            stored.append(regs[int(args[0][1:])].copy())
            continue
        if op == "ds_write_b32":
            v = regs[int(args[1].split()[0][1:])]
            for l in range(lanes):
                lds[lds_index(rest, l)] = v[l]
            continue
        if op == "ds_read_b32":
            d = int(args[0][1:])
            regs[d] = np.array([lds[lds_index(rest, l)] for l in range(lanes)], dtype=np.uint32)
            continue
        if op == "ds_read_b128":
            lo, hi = (int(x) for x in re.match(r"v\[(\d+):(\d+)\]", args[0]).groups())
            for k in range(4):
                regs[lo + k] = np.array([lds[lds_index(rest, l) + k] for l in range(lanes)], dtype=np.uint32)
            continue
        if op == "buffer_store_dwordx4":
            lo = int(re.match(r"v\[(\d+):", args[0]).group(1))
            for q in range(4):  # clock q of the group: lane 4j+q holds slice 4j+k's word in register lo+k
                stored.append(np.array([regs[lo + l % 4][l - l % 4 + q] for l in range(lanes)], dtype=np.uint32))
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


def written_before_read(insts, homes):
    """True if every register an instruction reads is a home register or was written by an
    earlier instruction of the body."""
    written = {v for v, _, _ in homes}
    for ins in insts:
        op, _, rest = ins.partition(" ")
        if op in ("buffer_store_dword", "ds_write_b32"):
            data = rest.split(",")[0 if op == "buffer_store_dword" else 1].strip().split()[0]
            if int(data[1:]) not in written:
                return False
            continue
        if op == "ds_read_b128":
            lo, hi = (int(x) for x in re.match(r"v\[(\d+):(\d+)\]", rest).groups())
            written.update(range(lo, hi + 1))
            continue
        if op == "ds_read_b32":
            written.add(int(rest.split(",")[0].strip()[1:]))
            continue
        if op == "buffer_store_dwordx4":
            lo, hi = (int(x) for x in re.match(r"v\[(\d+):(\d+)\]", rest).groups())
            if any(r not in written for r in range(lo, hi + 1)):
                return False
            continue
        if not op.startswith("v_"):
            continue
        regs = [int(x.strip().split()[0][1:]) for x in rest.split(",")]
        if any(src not in written for src in regs[1:]):
            return False
        written.add(regs[0])
    return True
