#!/usr/bin/env python3
"""Writes grain_clock_loop.inc: 80 clocks of the bitsliced Grain v1 keystream loop (one
revolution of the register rings) as one inline-assembly block, with every VGPR placed for
gfx950's register banks.

Why: a v_bitop3_b32 whose sources include two different VGPRs of one bank (register index
mod 4) issues at about half rate on MI355X; the compiler's allocation of the Grain loop had
2351 such instructions per 160 clocks (~15 per 36-op clock).

How.  The 80 NFSR words b and 80 LFSR words s are rings: after clock t the oldest bit sits
in slot t mod 80 and the clock's new bits overwrite that slot, so tap b_k of clock t is slot
(t + k) mod 80 (grain_bitslice.h).  A tap pair that shares an instruction is therefore at a
fixed slot distance in every clock, and whether it clashes depends only on the bank given
to each slot.  BANK_B / BANK_S below give each slot its bank (found by a search that
minimises clashes over all 80 rotations, together with GROUPING, the grouping of the three
free XOR sums into three-input XORs).  Temporaries take registers whose banks differ from
their co-sources where possible.  The ops are then list-scheduled under every register
order (read-after-write at distance LAT, write-after-read, write-after-write).

The clock is the one of grain_bitslice.h (36 VALU per 32 instances, generation mode):
  z   = b1^b2^b4^b10^b31^b43^b56 ^ h(s3, s25, s46, s64, b63), h = A ^ (x2 & B),
        A = x1 ^ f(x0,x3,x4), B = (x3 & ~(x0^x4)) ^ MAJ(x0,x1,x4)
  s80 = s0^s13^s23^s38^s51^s62
  b80 = s0 ^ g(b) with the monomials built from the shared pair products of that header.

Run from this directory: python3 gen_grain_loop.py  (rewrites grain_clock_loop.inc).
"""
from __future__ import annotations

import os

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "grain_clock_loop.inc")

TA, TB, TC = 0xF0, 0xCC, 0xAA
K_XOR3 = TA ^ TB ^ TC
K_AND3 = TA & TB & TC
K_XORAND = (TA ^ (TB & TC)) & 0xFF
K_F = (TC ^ (TA & TB) ^ (TB & TC)) & 0xFF                 # (x0, x3, x4)
K_MAJ = ((TA & TB) | (TA & TC) | (TB & TC)) & 0xFF       # (x0, x1, x4)
K_B = ((TA & (TB ^ 0xFF)) ^ TC) & 0xFF                    # (x3, x0^x4, maj)
RING = 80
LAT = 8
RESERVED = (0, 1, 2, 3)  # left to the compiler (the lane offset lives there)

# Bank of ring slot j (b ring, s ring) and the grouping of the free XOR sums (indices into
# the term lists below, taken three at a time), from the clash search.
BANK_B = [0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2,
          1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3]
BANK_S = [1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3,
          0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2, 1, 3, 0, 0, 2, 1, 3, 3, 0, 2, 1, 1, 3, 0, 2, 2]
GROUPING = {"a": [5, 1, 4, 8, 7, 2, 3, 0, 6], "fs": [3, 5, 1, 2, 0, 4], "glin": [8, 2, 9, 6, 0, 3, 7, 5, 1, 11, 10, 4]}

A_TERMS = [("b", 1), ("b", 2), ("b", 4), ("b", 10), ("b", 31), ("b", 43), ("b", 56), ("s", 25), ("t", "f")]
FS_TERMS = [("s", 0), ("s", 13), ("s", 23), ("s", 38), ("s", 51), ("s", 62)]
GLIN_TERMS = [("s", 0), ("b", 62), ("b", 60), ("b", 52), ("b", 45), ("b", 37), ("b", 33), ("b", 28), ("b", 21),
              ("b", 14), ("b", 9), ("b", 0)]


class Op:
    __slots__ = ("kind", "text", "dst", "srcs")

    def __init__(self, kind, text, dst, srcs):
        self.kind, self.text, self.dst, self.srcs = kind, text, dst, list(srcs)


def ring_registers():
    """Physical registers of the two rings with the chosen banks, and the rest (temps)."""
    pool = {b: [r for r in range(256) if r % 4 == b and r not in RESERVED] for b in range(4)}
    rb = [pool[BANK_B[j]].pop(0) for j in range(RING)]
    rs = [pool[BANK_S[j]].pop(0) for j in range(RING)]
    temps = sorted(r for b in range(4) for r in pool[b])
    return rb, rs, temps


def clock_ops(R):
    """The clock with the oldest bit in slot R, as symbolic ops (dst, kind, imm, srcs).
    Sources: ("b", k) / ("s", k) taps, or temp names.  Destinations: temp names, or
    ("B", R) / ("S", R) for the ring slot the new bit goes to."""
    ops = []

    def op(dst, kind, srcs, imm=None):
        ops.append((dst, kind, imm, srcs))

    def tree(name, terms, grouping, final_dst):
        groups = [[terms[i] for i in grouping[k:k + 3]] for k in range(0, len(grouping) - len(grouping) % 3, 3)]
        rest = [terms[i] for i in grouping[len(grouping) - len(grouping) % 3:]]
        parts = []
        for k, g in enumerate(groups):
            op("%s%d" % (name, k), "b3", g, K_XOR3)
            parts.append("%s%d" % (name, k))
        parts += rest
        return parts

    op("f", "b3", [("s", 3), ("s", 64), ("b", 63)], K_F)
    op("m", "xor", [("s", 3), ("b", 63)])
    op("mj", "b3", [("s", 3), ("s", 25), ("b", 63)], K_MAJ)
    op("bb", "b3", [("s", 64), "m", "mj"], K_B)
    ap = tree("a", A_TERMS_T, GROUPING["a"], None)
    op("a", "b3", ap, K_XOR3)
    op("z", "b3", ["a", ("s", 46), "bb"], K_XORAND)
    op(None, "store", ["z"])
    fp = tree("fs", FS_TERMS, GROUPING["fs"], None)
    op("p1", "and", [("b", 63), ("b", 60)])
    op("p2", "and", [("b", 37), ("b", 33)])
    op("p3", "and", [("b", 15), ("b", 9)])
    op("p4", "and", [("b", 52), ("b", 45)])
    op("p5", "and", [("b", 28), ("b", 21)])
    op("m5", "and", [("b", 33), "p5"])
    op("t6", "b3", [("b", 63), ("b", 45), ("b", 28)], K_AND3)
    op("m7", "b3", [("b", 60), ("b", 52), "p2"], K_AND3)
    op("m8", "b3", ["p1", ("b", 21), ("b", 15)], K_AND3)
    op("m9", "b3", ["p1", "p4", ("b", 37)], K_AND3)
    op("m11", "b3", ["p4", "p2", "p5"], K_AND3)
    gp = tree("gl", GLIN_TERMS, GROUPING["glin"], None)
    op("g5", "b3", ["p1", "p2", "p3"], K_XOR3)
    op("g6", "b3", ["m5", "m7", "m8"], K_XOR3)
    op("g7", "xor", ["m9", "m11"])
    op("x1", "b3", gp[0:3], K_XOR3)
    op("q1", "b3", ["x1", ("b", 60), "p4"], K_XORAND)
    op("x2", "b3", [gp[3], "g5", "g6"], K_XOR3)
    op("q2", "b3", ["x2", "t6", ("b", 9)], K_XORAND)
    op("q3", "b3", ["g7", "m5", "p3"], K_XORAND)
    # the new bits go to the clock's oldest slots once every read of s_0 and b_0 is done
    op(("S", R), "xor", fp)
    op(("B", R), "b3", ["q1", "q2", "q3"], K_XOR3)
    return ops


A_TERMS_T = [t if t[0] != "t" else t[1] for t in A_TERMS]


def build():
    rb, rs, temps = ring_registers()
    out = []
    free = list(temps)  # FIFO: a freed register is reused as late as possible
    live = {}           # temp name -> register (per clock)
    for R in range(RING):
        sym = clock_ops(R)
        # last use of every temp within the clock
        last = {}
        for k, (dst, kind, imm, srcs) in enumerate(sym):
            for s in srcs:
                if isinstance(s, str):
                    last[s] = k
        # co-source banks per temp (ring sources only; temps are resolved as allocated)
        def reg_of(s):
            if isinstance(s, tuple):
                ring, k = s
                return (rb if ring == "b" else rs)[(R + k) % RING]
            return live[s]
        for k, (dst, kind, imm, srcs) in enumerate(sym):
            regs = [reg_of(s) for s in srcs]
            if dst is None:
                out.append(Op("store", "buffer_store_dword v%d, %%[voff], s[20:23], 0 offen" % regs[0], None, regs))
                out.append(Op("salu", "s_add_u32 s20, s20, %[pitch]\n\ts_addc_u32 s21, s21, 0", None, []))
            else:
                if isinstance(dst, tuple):
                    d = (rb if dst[0] == "B" else rs)[R]
                else:
                    # banks to avoid: those of the other sources of this temp's 3-source consumers
                    avoid = set()
                    for dst2, kind2, imm2, srcs2 in sym[k + 1:]:
                        if kind2 == "b3" and dst in srcs2:
                            for s2 in srcs2:
                                if s2 != dst and (isinstance(s2, tuple) or s2 in live):
                                    avoid.add(reg_of(s2) % 4)
                    pick = next((i for i, r in enumerate(free) if r % 4 not in avoid), 0)
                    d = free.pop(pick)
                    live[dst] = d
                if kind == "b3":
                    out.append(Op("valu", "v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (d, *regs, imm), d, regs))
                elif kind == "xor":
                    out.append(Op("valu", "v_xor_b32 v%d, v%d, v%d" % (d, *regs), d, regs))
                else:
                    out.append(Op("valu", "v_and_b32 v%d, v%d, v%d" % (d, *regs), d, regs))
            # free temps whose last use was this op
            for s in dict.fromkeys(x for x in srcs if isinstance(x, str)):  # in source order
                if last.get(s) == k:
                    free.append(live.pop(s))
        assert not live, live
    return out, rb, rs


def schedule(ops):
    n = len(ops)
    preds = [[] for _ in range(n)]
    last_w, reads = {}, {}
    prev_mem = None
    for k, o in enumerate(ops):
        for s in o.srcs:
            if s in last_w:
                preds[k].append((last_w[s], LAT if ops[last_w[s]].kind == "valu" else 1))
        if o.dst is not None:
            for r in reads.get(o.dst, []):
                preds[k].append((r, 1))
            if o.dst in last_w:
                preds[k].append((last_w[o.dst], 1))
        if o.kind in ("store", "salu"):
            if prev_mem is not None:
                preds[k].append((prev_mem, 1))
            prev_mem = k
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
    ops, rb, rs = build()
    sched = schedule(ops)
    nvalu = sum(o.kind == "valu" for o in sched)
    body = "\n\t".join(o.text.replace("\n", "\n\t") for o in sched)
    ring_regs = set(rb) | set(rs)
    used = sorted({r for o in ops for r in list(o.srcs) + ([o.dst] if o.dst is not None else [])})
    clob = [r for r in used if r not in ring_regs]
    out = ["// Generated by gen_grain_loop.py (the clock of grain_bitslice.h); do not edit.",
           "// %d clocks per iteration, %d VALU (%.1f per clock), %d bitop3 bank clashes."
           % (RING, nvalu, nvalu / RING, clashes(sched)),
           "#define GRAIN_LOOP_CLOCKS %d" % RING,
           "#define GRAIN_LOOP_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t"),
           "#define GRAIN_LOOP_STATE(B, S) \\\n    %s" % ", \\\n    ".join(
               ['"+{v%d}"(B(%d))' % (rb[j], j) for j in range(RING)] + ['"+{v%d}"(S(%d))' % (rs[j], j) for j in range(RING)]),
           "#define GRAIN_LOOP_CLOBBERS %s" % ", ".join('"v%d"' % r for r in clob)]
    return "\n".join(out) + "\n"


def main():
    text = render()
    with open(OUT, "w") as f:
        f.write(text)
    print(text.split("\n")[1])


if __name__ == "__main__":
    main()
