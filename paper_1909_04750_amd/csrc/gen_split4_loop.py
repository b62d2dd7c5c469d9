#!/usr/bin/env python3
"""Writes mickey_split4_loop.inc: the four-wave split keystream loop (two clocks per
iteration) for each of the four roles, as inline-assembly bodies with VGPRs placed for
gfx950's register banks (see gen_clock_loop.py for why).

The split (mickey_device.h): one workgroup of four waves serves 64 slices; wave 0 keeps
r_0..r_49, wave 1 r_50..r_99, wave 2 s_0..s_49, wave 3 s_50..s_99.  Every clock each wave
computes the next-state values the others need, writes them to a double-buffered LDS slot,
passes the clock's one barrier, reads what it needs for the next clock, and computes the
rest of its half.  Exchanged (next-state values): r_49, r_33 (wave 0); r_99, r_67 (wave 1);
s_49, s_34, s_0 (wave 2); s_50, s_99, s_67 (wave 3); wave 0 also stores the keystream word
z = r_0 ^ s_0 of every clock.  The LDS layout (slot order, buffer per clock parity) is the
one of Split4Lds, so that the C++ code before and after the loop (state load, first
exchange, an odd last clock, state store) is unchanged.

Registers: each wave keeps its 50 words in two sets (the update is functional: clock t reads
one set and writes the other, and two clocks per iteration return to the first), each set
in consecutive VGPRs, so s_{i-1}, s_i, s_{i+1} (and r_{i-1}, r_i) sit in different banks; c_R
is formed twice, in banks 0 and 2, and each R update takes the copy whose bank differs from
its other two sources; the imported words alternate between two register sets as well, and
an import that meets two state words in one instruction gets a bank apart from both.  Each
region between barriers is list-scheduled under every register order, with LDS reads LDS_LAT
instructions ahead of their first use (a s_waitcnt lgkmcnt(0) is placed before that use).

Run from this directory: python3 gen_split4_loop.py  (rewrites mickey_split4_loop.inc).
"""
from __future__ import annotations

import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mickey_split4_loop.inc")

TA, TB, TC = 0xF0, 0xCC, 0xAA
IMM_R = (TA ^ (TB & TC)) & 0xFF
LAT = 6
LDS_LAT = 16
SLOTS = ["R49", "R33", "R99", "R67", "S49", "S34", "S0", "S50", "S99", "S67"]  # Split4Lds order
NSLOT = len(SLOTS)
SET_A, SET_B = 4, 56  # first VGPR of each 50-word state set (banks follow the position)
# imports and temporaries; v0-v3 are left to the compiler, and the whole body stays within
# the 128 VGPRs of four waves per SIMD
POOL = [54, 55] + list(range(106, 128))

# role: (register, first position, imports (name, C++ binding), exports (position, slot))
ROLES = [
    ("r", 0, [("r99", "in.a"), ("r67", "in.b"), ("s34", "in.c"), ("s0", "in.d")], [(49, "R49"), (33, "R33")]),
    ("r", 50, [("r49", "x.r[49]"), ("s34", "in.a")], [(99, "R99"), (67, "R67")]),
    ("s", 0, [("s50", "x.s[50]"), ("s99", "in.a"), ("s67", "in.b"), ("r33", "in.c")], [(49, "S49"), (34, "S34"), (0, "S0")]),
    ("s", 50, [("s49", "x.s[49]"), ("r33", "in.a")], [(50, "S50"), (99, "S99"), (67, "S67")]),
]
SLOT_OF_IMPORT = {"r99": "R99", "r67": "R67", "s34": "S34", "s0": "S0", "r49": "R49", "s50": "S50", "s99": "S99",
                  "s67": "S67", "r33": "R33", "s49": "S49"}


def tables():
    src = open(os.path.join(HERE, "mickey_bitslice.h")).read()

    def arr(name):
        m = re.search(r"constexpr uint8_t %s\[\] = \{([^}]*)\};" % name, src)
        return {int(x) for x in m.group(1).replace("\n", " ").split(",") if x.strip()}
    return {n: arr(n) for n in ("kRTaps", "kComp0", "kComp1", "kFb0", "kFb1")}


class Op:
    __slots__ = ("kind", "text", "dsts", "srcs")

    def __init__(self, kind, text, dsts, srcs):
        self.kind, self.text, self.dsts, self.srcs = kind, text, list(dsts), list(srcs)


def role_body(role, tab):
    reg, j0, imports, exports = ROLES[role]
    own = range(j0, j0 + 50)
    sets = [{j0 + k: SET_A + k for k in range(50)}, {j0 + k: SET_B + k for k in range(50)}]
    # import registers (two sets), temporaries, keystream word
    pool = list(POOL)

    def take(avoid=()):
        for k, v in enumerate(pool):
            if v % 4 not in avoid:
                return pool.pop(k)
        return pool.pop(0)

    def import_avoid(name):
        # banks of the state words an import meets inside one bitop3
        if name == "r49":   # r_50 <- r_49 ^ (c & r_50)
            return {sets[0][50] % 4, sets[1][50] % 4}
        if name == "s50":   # s_49 <- f(s_48, s_49, s_50)
            return {sets[0][48] % 4, sets[0][49] % 4, sets[1][48] % 4, sets[1][49] % 4}
        if name == "s49":   # s_50 <- f(s_49, s_50, s_51)
            return {sets[0][50] % 4, sets[0][51] % 4, sets[1][50] % 4, sets[1][51] % 4}
        return set()
    imp = [{}, {}]
    for name, _ in imports:
        for p in (0, 1):
            imp[p][name] = take(import_avoid(name))
    # per clock parity, so that the next clock's control bits do not wait for the current
    # clock's last reader
    ctl = [(take(avoid=(1, 2, 3)), take(avoid=(0, 1, 3)), take(), take(), take()) for _ in (0, 1)]
    # the wave that owns position 99 reads the feedback bit from a copy: the next clock's
    # export of that position then need not wait for the current clock's last tap
    fb_copy = [take(), take()] if 99 in own else None
    zreg = take()
    regions = [[], [], []]  # before barrier 1 | between barriers | after barrier 2

    def emit(region, kind, text, dsts, srcs):
        regions[region].append(Op(kind, text, dsts, srcs))

    def v3(region, dst, a, b, c, imm):
        emit(region, "valu", "v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (dst, a, b, c, imm), [dst], [a, b, c])

    def v2(region, name, dst, a, b):
        emit(region, "valu", "%s v%d, v%d, v%d" % (name, dst, a, b), [dst], [a, b])

    for t in (0, 1):
        cur, nxt = sets[t], sets[1 - t]
        im, im_next = imp[t], imp[1 - t]
        cra, crb, cs, g0, g1 = ctl[t]
        ph = 1 - t                     # clock t writes exchange buffer (t + 1) & 1
        pre, post = t, t + 1           # region before this clock's barrier, region after it

        def src_of(name):
            if name in im:
                return im[name]
            return cur[int(name[1:])]

        if reg == "r":
            fbr = src_of("r99")
            if fb_copy:
                emit(pre, "valu", "v_mov_b32 v%d, v%d" % (fb_copy[t], fbr), [fb_copy[t]], [fbr])
                fbr = fb_copy[t]
            v2(pre, "v_xor_b32", cra, src_of("s34"), src_of("r67"))
            v2(pre, "v_xor_b32", crb, src_of("s34"), src_of("r67"))
            if role == 0:  # keystream word of the current state
                v2(pre, "v_xor_b32", zreg, cur[0], im["s0"])
                emit(pre, "store", "buffer_store_dword v%d, %%[voff], s[20:23], 0 offen" % zreg, [], [zreg])
                emit(pre, "salu", "s_add_u32 s20, s20, %[pitch]\n\ts_addc_u32 s21, s21, 0", [], [])

            def r_update(i, region):
                a = fbr if i == 0 else (cur[i - 1] if i - 1 in own else src_of("r%d" % (i - 1)))
                b = cur[i]
                c = cra if cra % 4 not in (a % 4, b % 4) else crb
                v3(region, nxt[i], a, c, b, IMM_R)
                if i != 0 and i in tab["kRTaps"]:
                    v2(region, "v_xor_b32", nxt[i], nxt[i], fbr)
            exp_pos = [p for p, _ in exports]
            for p in exp_pos:
                r_update(p, pre)
            for i in own:
                if i not in exp_pos:
                    r_update(i, post)
        else:
            fbs = src_of("s99")
            if fb_copy:
                emit(pre, "valu", "v_mov_b32 v%d, v%d" % (fb_copy[t], fbs), [fb_copy[t]], [fbs])
                fbs = fb_copy[t]
            v2(pre, "v_xor_b32", cs, src_of("s67"), src_of("r33"))
            v2(pre, "v_and_b32", g1, fbs, cs)
            v2(pre, "v_xor_b32", g0, fbs, g1)

            def sel_of(i):
                f0, f1 = i in tab["kFb0"], i in tab["kFb1"]
                return fbs if (f0 and f1) else g0 if f0 else g1 if f1 else None

            def s_update(i, region):
                if i == 0:
                    emit(region, "valu", "v_mov_b32 v%d, v%d" % (nxt[0], fbs), [nxt[0]], [fbs])
                    return
                if i == 99:
                    v2(region, "v_xor_b32", nxt[99], cur[98], sel_of(99))
                    return
                a = cur[i - 1] if i - 1 in own else src_of("s%d" % (i - 1))
                c = cur[i + 1] if i + 1 in own else src_of("s%d" % (i + 1))
                bb = (TB ^ 0xFF) if i in tab["kComp0"] else TB
                cc = (TC ^ 0xFF) if i in tab["kComp1"] else TC
                v3(region, nxt[i], a, cur[i], c, (TA ^ (bb & cc)) & 0xFF)
                if sel_of(i) is not None:
                    v2(region, "v_xor_b32", nxt[i], nxt[i], sel_of(i))
            exp_pos = [p for p, _ in exports]
            for p in exp_pos:
                s_update(p, pre)
            for i in own:
                if i not in exp_pos:
                    s_update(i, post)
        # exports, barrier, imports for the next clock
        for p, slot in exports:
            off = (ph * NSLOT + SLOTS.index(slot)) * 256
            emit(pre, "ldsw", "ds_write_b32 %%[xaddr], v%d offset:%d" % (nxt[p], off), [], [nxt[p]])
        emit(pre, "barrier", "s_waitcnt lgkmcnt(0)\n\ts_barrier", [], [])
        for name, _ in imports:
            off = (ph * NSLOT + SLOTS.index(SLOT_OF_IMPORT[name])) * 256
            emit(post, "ldsr", "ds_read_b32 v%d, %%[xaddr] offset:%d" % (im_next[name], off), [im_next[name]], [])
    # the imports read after the second barrier are the next iteration's first inputs
    emit(2, "wait", "s_waitcnt lgkmcnt(0)", [], [])
    home_state = sets[0]
    home_imp = imp[0]
    used = {r for rg in regions for o in rg for r in o.dsts + o.srcs}
    clob = sorted(used - set(home_state.values()) - set(home_imp.values()))
    return regions, home_state, home_imp, clob


def schedule(ops):
    """List-schedule one region; the barrier (if any) stays last.  Returns texts, with a
    s_waitcnt lgkmcnt(0) before the first use of each LDS-read register."""
    tail = [o for o in ops if o.kind in ("barrier", "wait")]
    ops = [o for o in ops if o.kind not in ("barrier", "wait")]
    n = len(ops)
    preds = [[] for _ in range(n)]
    last_w, reads = {}, {}
    prev = {}
    for k, o in enumerate(ops):
        for s in o.srcs:
            if s in last_w:
                w = ops[last_w[s]].kind
                preds[k].append((last_w[s], LDS_LAT if w == "ldsr" else LAT if w == "valu" else 1))
        for d in o.dsts:
            for r in reads.get(d, []):
                preds[k].append((r, 1))
            if d in last_w:
                preds[k].append((last_w[d], 1))
        cls = "lds" if o.kind in ("ldsw", "ldsr") else "mem" if o.kind in ("store", "salu") else None
        if cls:
            if cls in prev:
                preds[k].append((prev[cls], 1))
            prev[cls] = k
        for s in o.srcs:
            reads.setdefault(s, []).append(k)
        for d in o.dsts:
            last_w[d] = k
            reads[d] = []
    succs = [[] for _ in range(n)]
    for k in range(n):
        for p, d in preds[k]:
            succs[p].append((k, d))
    # LDS writes, and everything that computes their data, go first: they gate the barrier
    height = [0] * n
    for k in range(n - 1, -1, -1):
        height[k] = max([height[s] + d for s, d in succs[k]] + [1000 if ops[k].kind == "ldsw" else 0])
    npred = [len(p) for p in preds]
    ready_at = [0] * n
    avail = [k for k in range(n) if npred[k] == 0]
    order, slot = [], 0
    while avail:
        cands = [k for k in avail if ready_at[k] <= slot] or avail
        k = max(cands, key=lambda j: (height[j], -j))
        avail.remove(k)
        order.append(k)
        for s, d in succs[k]:
            ready_at[s] = max(ready_at[s], slot + d)
            npred[s] -= 1
            if npred[s] == 0:
                avail.append(s)
        slot += 1
    out = []
    pending = set()
    for k in order:
        o = ops[k]
        if pending & set(o.srcs):
            out.append("s_waitcnt lgkmcnt(0)")
            pending = set()
        out.append(o.text)
        if o.kind == "ldsr":
            pending |= set(o.dsts)
    return out + [o.text for o in tail]


def clashes(texts):
    bad = 0
    for t in texts:
        if t.startswith("v_bitop3"):
            regs = sorted({int(x) for x in re.findall(r"v(\d+)", t)[1:4]})
            banks = [r % 4 for r in regs]
            bad += len(banks) - len(set(banks))
    return bad


def render() -> str:
    tab = tables()
    out = ["// Generated by gen_split4_loop.py from the tables of mickey_bitslice.h; do not edit."]
    for role in range(4):
        regions, home_state, home_imp, clob = role_body(role, tab)
        texts = []
        for rg in regions:
            texts += schedule(rg)
        nvalu = sum(1 for t in texts if t.startswith("v_"))
        reg, j0, imports, _ = ROLES[role]
        body = "\n\t".join(t.replace("\n", "\n\t") for t in texts)
        out.append("// role %d (%s_%d..%s_%d): %d VALU per 2 clocks, %d bitop3 bank clashes"
                   % (role, reg, j0, reg, j0 + 49, nvalu, clashes(texts)))
        out.append("#define MICKEY_S4_BODY_%d \\\n    \"%s\\n\"" % (role, body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t")))
        ops_list = ['"+{v%d}"(%s.%s[%d].w[0])' % (home_state[p], "x", reg, p) for p in sorted(home_state)]
        ops_list += ['"+{v%d}"(%s.w[0])' % (home_imp[name], binding) for name, binding in imports]
        out.append("#define MICKEY_S4_STATE_%d \\\n    %s" % (role, ", \\\n    ".join(ops_list)))
        out.append("#define MICKEY_S4_CLOBBERS_%d %s" % (role, ", ".join('"v%d"' % r for r in clob)))
    return "\n".join(out) + "\n"


def main():
    text = render()
    with open(OUT, "w") as f:
        f.write(text)
    for line in text.split("\n"):
        if line.startswith("// role"):
            print(line)


if __name__ == "__main__":
    main()
