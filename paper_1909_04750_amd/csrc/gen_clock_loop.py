#!/usr/bin/env python3
"""Writes mickey_clock_loop.inc: the bitsliced MICKEY 2.0 keystream loop body as one
inline-assembly block with a register assignment chosen for gfx950's VGPR banks.

Why: a v_bitop3_b32 whose three sources include two different VGPRs of the same bank
(register index mod 4) issues at about half rate on MI355X, and the compiler's register
allocator does not know it (the compiled generate loop had 551 such clashes among its
891 bitop3 per 4 clocks).  Here every register is placed by this script:

- R words live in v[R0 .. R0+99] (r_i in R0+i, except that r_99 alternates with a spare
  register from clock to clock), S words in a ring of 100 registers whose origin moves by
  one per clock (an ascending in-place sweep leaves the new s_i where the old s_{i-1}
  was); two clocks per loop iteration, ascending then descending, return every word to
  its register, so the loop needs no copies;
- the control bit c_R is formed twice, in banks 0 and 2, and each R update reads the copy
  whose bank differs from both of its other sources (r_{i-1} and r_i are neighbours);
- the S sources s_{i-1}, s_i, s_{i+1} sit in consecutive registers of the ring, hence in
  three different banks;
- the instructions are then list-scheduled (respecting every read-after-write,
  write-after-read and write-after-write order on the assigned registers) so that a
  result is consumed no sooner than LAT instructions after it is produced.

The clock itself is the one of mickey_bitslice.h (whose tables are parsed from that
header), per 32 instances: c_R = s_34 ^ r_67, c_S = s_67 ^ r_33, g1 = s_99 & c_S,
g0 = s_99 ^ g1; r_i <- r_{i-1} ^ (c_R & r_i) (^ r_99 at the feedback taps); s_i <- s_{i-1}
^ ((s_i ^ C0_i) & (s_{i+1} ^ C1_i)) (^ g0 / g1 / s_99 where FB0_i / FB1_i select it);
s_0 <- s_99; and before each clock the keystream word z = r_0 ^ s_0 is stored.

Run from this directory: python3 gen_clock_loop.py  (rewrites mickey_clock_loop.inc).
"""
from __future__ import annotations

import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mickey_clock_loop.inc")
OUT_MIX = os.path.join(HERE, "mickey_mix_loop.inc")

TA, TB, TC = 0xF0, 0xCC, 0xAA
N = 100
CLOCKS = 2       # clocks per loop iteration (ascending, then descending S sweep)
LAT = 8          # minimum distance, in VALU instructions, from a result to its first use
R0 = 8           # r_i in v[R0 + i]
S0 = 112         # the S ring: v[S0 .. S0 + 99]
SPARE_R = 108    # r_99 of odd clocks
TEMPS = list(range(212, 256)) + list(range(4, 8)) + [109, 110, 111]  # c_R copies, c_S, g0, g1, z
MIX_IN = [4, 5]  # the mixing body's input words (clock 0, clock 1 of the pair)


def tables():
    src = open(os.path.join(HERE, "mickey_bitslice.h")).read()

    def arr(name):
        m = re.search(r"constexpr uint8_t %s\[\] = \{([^}]*)\};" % name, src)
        return {int(x) for x in m.group(1).replace("\n", " ").split(",") if x.strip()}
    return {n: arr(n) for n in ("kRTaps", "kComp0", "kComp1", "kFb0", "kFb1")}


class Op:
    __slots__ = ("text", "dst", "srcs", "kind", "n")

    def __init__(self, kind, text, dst, srcs):
        self.kind, self.text, self.dst, self.srcs = kind, text, dst, list(srcs)


def build(tab, mix=False):
    """The CLOCKS-clock body as ops on physical registers, in program order.  With mix, the
    initialisation clock instead (CLOCK_KG with mixing on, input word MIX_IN[t] of the
    pair): fb_R = r_99 ^ in ^ s_50 and fb_S = s_99 ^ in in temporaries, the new s_0 (= fb_S)
    moved into the register the ring gives it, and no keystream store."""
    ops = []
    rr = {i: R0 + i for i in range(N)}          # where r_i lives
    ring = [S0 + i for i in range(N)]           # where s_i lives: ring[i]
    zregs = [TEMPS[0], TEMPS[1]]                # keystream words, one per clock of the pair
    free_temps = [t for t in TEMPS if t not in zregs and not (mix and t in MIX_IN)]

    def take(avoid_banks=()):
        for k, v in enumerate(free_temps):
            if v % 4 not in avoid_banks:
                return free_temps.pop(k)
        return free_temps.pop(0)

    def v3(dst, a, b, c, imm):
        ops.append(Op("valu", "v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (dst, a, b, c, imm), dst, (a, b, c)))

    def v2(name, dst, a, b):
        ops.append(Op("valu", "%s v%d, v%d, v%d" % (name, dst, a, b), dst, (a, b)))

    def pick_c(cra, crb, a, b):
        for c in (cra, crb):
            if c % 4 not in (a % 4, b % 4):
                return c
        return cra

    spare_r = SPARE_R
    for t in range(CLOCKS):
        ascending = t % 2 == 0
        if not mix:
            # keystream word of the current state, and its store (plane address advanced by SALU)
            z = zregs[t % 2]
            v2("v_xor_b32", z, rr[0], ring[0])
            ops.append(Op("store", "buffer_store_dword v%d, %%[voff], s[20:23], 0 offen" % z, None, (z,)))
            ops.append(Op("salu", "s_add_u32 s20, s20, %[pitch]\n\ts_addc_u32 s21, s21, 0", None, ()))
        # control bits and feedback selections
        cra, crb = take(avoid_banks=(1, 2, 3)), take(avoid_banks=(0, 1, 3))
        v2("v_xor_b32", cra, ring[34], rr[67])
        v2("v_xor_b32", crb, ring[34], rr[67])
        cs = take()
        v2("v_xor_b32", cs, ring[67], rr[33])
        old_s99, old_r99 = ring[99], rr[99]
        if mix:
            fbs = take()
            v2("v_xor_b32", fbs, ring[99], MIX_IN[t])
            fbr = take()
            v3(fbr, rr[99], MIX_IN[t], ring[50], 0x96)
        else:
            fbs, fbr = ring[99], rr[99]
        g1 = take()
        v2("v_and_b32", g1, fbs, cs)
        g0 = take()
        v2("v_xor_b32", g0, fbs, g1)
        free_temps.append(cs)
        # R sweep, descending, in place; r_99 goes to the spare (old r_99 is read by the
        # feedback and by its own update)
        imm_r = (TA ^ (TB & TC)) & 0xFF
        for i in range(N - 1, -1, -1):
            if i == 0:
                v3(rr[0], fbr, pick_c(cra, crb, fbr, rr[0]), rr[0], imm_r)
                continue
            a, b = rr[i - 1], rr[i]
            dst = spare_r if i == N - 1 else b
            v3(dst, a, pick_c(cra, crb, a, b), b, imm_r)
            if i in tab["kRTaps"]:
                v2("v_xor_b32", dst, dst, fbr)
        rr[N - 1], spare_r = spare_r, old_r99  # old r_99's register is free after the sweep
        free_temps += [cra, crb]
        if mix:
            free_temps.append(fbr)

        # S sweep
        def sel_of(i):
            f0, f1 = i in tab["kFb0"], i in tab["kFb1"]
            return fbs if (f0 and f1) else g0 if f0 else g1 if f1 else None

        def s_update(i, a, b, c, dst):
            bb = (TB ^ 0xFF) if i in tab["kComp0"] else TB
            cc = (TC ^ 0xFF) if i in tab["kComp1"] else TC
            v3(dst, a, b, c, (TA ^ (bb & cc)) & 0xFF)
            if sel_of(i) is not None:
                v2("v_xor_b32", dst, dst, sel_of(i))

        assert sel_of(N - 1) is not None, "the s_99 update is one op"
        if ascending:
            # new s_i where old s_{i-1} was (it dies at that op), new s_99 where old s_98 was;
            # new s_0 is the old s_99 (the feedback word), renamed
            for i in range(1, N - 1):
                s_update(i, ring[i - 1], ring[i], ring[i + 1], ring[i - 1])
            v2("v_xor_b32", ring[N - 2], ring[N - 2], sel_of(N - 1))
            ring = [ring[N - 1]] + ring[:N - 1]
        else:
            # old s_99 stays (feedback, then new s_0); new s_99 and s_98 go to temporaries,
            # new s_i (i <= 97) where old s_{i+1} was; old s_0 and s_1 end up free
            t99, t98 = take(), take()
            v2("v_xor_b32", t99, ring[N - 2], sel_of(N - 1))
            s_update(N - 2, ring[N - 3], ring[N - 2], ring[N - 1], t98)
            for i in range(N - 3, 0, -1):
                s_update(i, ring[i - 1], ring[i], ring[i + 1], ring[i + 1])
            freed = [ring[0], ring[1]]
            ring = [ring[N - 1]] + ring[2:N - 1] + [t98, t99]
            free_temps += freed
        if mix:
            # the new s_0 is fb_S; the ring gives it the old s_99's register
            assert ring[0] == old_s99
            ops.append(Op("valu", "v_mov_b32 v%d, v%d" % (old_s99, fbs), old_s99, (fbs,)))
            free_temps.append(fbs)
        free_temps += [g0, g1]
    # return every S word to its home register (a parallel move over the displaced ones)
    home = [S0 + i for i in range(N)]
    pending = {home[i]: ring[i] for i in range(N) if ring[i] != home[i]}  # dst <- src
    while pending:
        srcs = set(pending.values())
        ready = [d for d in pending if d not in srcs]
        assert ready, "cyclic fix-up needs a temporary"
        for d in ready:
            ops.append(Op("valu", "v_mov_b32 v%d, v%d" % (d, pending[d]), d, (pending[d],)))
            del pending[d]
    ring = home
    return ops, rr, ring


def schedule(ops):
    """List scheduling under RAW (LAT), WAR and WAW orders on physical registers."""
    n = len(ops)
    preds = [[] for _ in range(n)]  # (pred, min distance)
    last_w, reads = {}, {}
    for k, o in enumerate(ops):
        for s in o.srcs:
            if s in last_w:
                preds[k].append((last_w[s], LAT if ops[last_w[s]].kind == "valu" else 1))
        if o.dst is not None:
            for r in reads.get(o.dst, []):
                preds[k].append((r, 1))
            if o.dst in last_w:
                preds[k].append((last_w[o.dst], 1))
        if o.kind in ("store", "salu"):  # stores stay in order with their address updates
            prev = [j for j in range(k) if ops[j].kind in ("store", "salu")]
            if prev:
                preds[k].append((prev[-1], 1))
        for s in o.srcs:
            reads.setdefault(s, []).append(k)
        if o.dst is not None:
            last_w[o.dst] = k
            reads[o.dst] = []
    succs = [[] for _ in range(n)]
    for k in range(n):
        for p, d in preds[k]:
            succs[p].append((k, d))
    height = [0] * n
    for k in range(n - 1, -1, -1):
        height[k] = max([height[s] + d for s, d in succs[k]] or [0])
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
    assert len(order) == n
    return [ops[k] for k in order]


def clashes(ops):
    bad = 0
    for o in ops:
        if o.text.startswith("v_bitop3"):
            regs = sorted(set(o.srcs))
            banks = [r % 4 for r in regs]
            bad += len(banks) - len(set(banks))
    return bad


def render() -> str:
    tab = tables()
    ops, rr, ring = build(tab)
    assert rr == {i: R0 + i for i in range(N)}, "R registers must return to their homes"
    assert ring == [S0 + i for i in range(N)], "the S ring must return to its origin"
    sched = schedule(ops)
    nvalu = sum(o.kind == "valu" for o in sched)
    body = "\n\t".join(o.text.replace("\n", "\n\t") for o in sched)
    used = sorted({r for o in ops for r in list(o.srcs) + ([o.dst] if o.dst is not None else [])})
    clob = [r for r in used if not (R0 <= r < R0 + N or S0 <= r < S0 + N)]
    out = ["// Generated by gen_clock_loop.py from the tables of mickey_bitslice.h; do not edit.",
           "// %d clocks per iteration, %d VALU (%.1f per clock), %d bitop3 bank clashes."
           % (CLOCKS, nvalu, nvalu / CLOCKS, clashes(sched)),
           "#define MICKEY_LOOP_CLOCKS %d" % CLOCKS,
           "#define MICKEY_LOOP_VALU %d" % nvalu,
           "#define MICKEY_LOOP_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t"),
           "#define MICKEY_LOOP_STATE(R, S) \\\n    %s" % ", \\\n    ".join(
               ['"+{v%d}"(R(%d))' % (R0 + i, i) for i in range(N)] + ['"+{v%d}"(S(%d))' % (S0 + i, i) for i in range(N)]),
           "#define MICKEY_LOOP_CLOBBERS %s" % ", ".join('"v%d"' % r for r in clob)]
    return "\n".join(out) + "\n"


def render_mix() -> str:
    tab = tables()
    ops, rr, ring = build(tab, mix=True)
    assert rr == {i: R0 + i for i in range(N)}, "R registers must return to their homes"
    assert ring == [S0 + i for i in range(N)], "the S ring must return to its origin"
    sched = schedule(ops)
    nvalu = sum(o.kind == "valu" for o in sched)
    body = "\n\t".join(o.text.replace("\n", "\n\t") for o in sched)
    used = sorted({r for o in ops for r in list(o.srcs) + ([o.dst] if o.dst is not None else [])})
    clob = [r for r in used if not (R0 <= r < R0 + N or S0 <= r < S0 + N) and r not in MIX_IN]
    out = ["// Generated by gen_clock_loop.py from the tables of mickey_bitslice.h; do not edit.",
           "// Initialisation (mixing) clocks: %d per body, %d VALU (%.1f per clock), %d bitop3 bank clashes."
           % (CLOCKS, nvalu, nvalu / CLOCKS, clashes(sched)),
           "#define MICKEY_MIX_CLOCKS %d" % CLOCKS,
           "#define MICKEY_MIX_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t"),
           "#define MICKEY_MIX_INPUTS(IN0, IN1) \"{v%d}\"(IN0), \"{v%d}\"(IN1)" % (MIX_IN[0], MIX_IN[1]),
           "#define MICKEY_MIX_CLOBBERS %s" % ", ".join('"v%d"' % r for r in clob)]
    return "\n".join(out) + "\n"


def main():
    text = render()
    with open(OUT, "w") as f:
        f.write(text)
    print(text.split("\n")[1])
    text = render_mix()
    with open(OUT_MIX, "w") as f:
        f.write(text)
    print(text.split("\n")[1])


if __name__ == "__main__":
    main()
