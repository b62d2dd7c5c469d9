#!/usr/bin/env python3
"""Writes mickey128_loops.inc: the keystream loops of m128_gen_kernel's two waves (MICKEY-128
2.0, two clocks per iteration) as inline-assembly bodies with VGPRs placed for gfx950's
register banks (gen_clock_loop.py explains the bank rule: a v_bitop3_b32 whose sources
include two different registers of one bank issues at about half rate) and, for the S
wave, list-scheduled so that no result is read sooner than LAT instructions after it is
produced (the compiled S loop read 54 results per 2 clocks in the very next instruction).

R wave:
The R wave keeps r_0..r_159 in place in v7..v166 and updates them in one descending sweep
per clock, r_i <- r_{i-1} ^ (c_R & r_i) (^ the feedback r_159 at the taps), r_0 <- fb ^
(c_R & r_0).  Per clock, in the order of r_gen_clock in mickey128_kernels.hip:
  - the old r_159 is copied (the feedback bit; r_159 is the first word the sweep rewrites);
  - c_R = s_54 ^ r_106 is formed twice, in banks 0 and 2: r_{i-1} and r_i sit in adjacent
    banks, so one of the two copies is always in a third bank;
  - the keystream word r_0 ^ s_0 of the state before the clock is formed in place in the
    s_0 register and stored through the buffer resource in s[20:23];
  - r_159 .. r_53 are updated, the new r_53 is written to the exchange slot of the clock's
    parity, and after the workgroup barrier the S wave's new s_54 and s_0 are read into
    their registers (the clock no longer needs the old ones);
  - r_52 .. r_0 are updated.
Tap XORs trail their position's update by a few instructions (the sweep's updates do not
depend on each other, the XOR depends on its update).  The LDS offsets follow XLds (r53,
s54, s0, s80, each [2][64] words); clock t writes parity (t + 1) & 1.

S wave: s_0..s_159 in a ring of 160 registers, in the way of gen_clock_loop.py.  Per
clock, as s_gen_clock in mickey128_kernels.hip: c_S = s_106 ^ r_53 (the R wave's word,
read after the previous clock's barrier), g1 = fb & c_S, g0 = fb ^ g1 with fb the old
s_159; the first clock of an iteration sweeps up (new s_i where old s_{i-1} was), the
second down (new s_i where old s_{i+1} was; new s_159 and s_158 in temporaries); in each,
once s_54 is new, it and the next s_0 (= fb) are written to the exchange slots, the
barrier passes, and the next r_53 is read.  A few moves at the end of the iteration put
every word back in its home register.  v2..v7 hold g0, g1, c_S (then the descending new
s_158), r_53, the descending new s_159 and a spare.

Run from this directory: python3 gen_m128_loop.py  (rewrites mickey128_loops.inc).
"""
from __future__ import annotations

import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mickey128_loops.inc")

N = 160
RB = 7                         # r_i in v(RB + i)
S54, S0, CRA, CRB, FBC = 3, 6, 4, 2, 5
assert CRA % 4 == 0 and CRB % 4 == 2 and FBC % 4 not in (CRA % 4, (RB + 0) % 4)
CTL_RR, CTL_SR = 106, 53       # c_R = s_54 ^ r_106; the S wave's control bit needs r_53
XOR_DELAY = 4
OFF_R53, OFF_S54, OFF_S0 = 0, 512, 1024
IMM_R = (0xF0 ^ (0xCC & 0xAA)) & 0xFF  # a ^ (b & c)


def tables():
    src = open(os.path.join(HERE, "mickey128_bitslice.h")).read()

    def arr(name):
        m = re.search(r"constexpr uint8_t %s\[\] = \{([^}]*)\};" % name, src)
        return {int(x) for x in m.group(1).replace("\n", " ").split(",") if x.strip()}
    return {n: arr(n) for n in ("kRTaps", "kComp0", "kComp1", "kFb0", "kFb1")}


def taps():
    return tables()["kRTaps"]


def r(i):
    return RB + i


def clock(tapset, ph):
    """Instructions of one clock that writes exchange parity `ph`."""
    out = ["v_mov_b32 v%d, v%d" % (FBC, r(N - 1)),
           "s_waitcnt lgkmcnt(0)",  # the imports read after the previous clock's barrier
           "v_xor_b32 v%d, v%d, v%d" % (CRA, S54, r(CTL_RR)),
           "v_xor_b32 v%d, v%d, v%d" % (CRB, S54, r(CTL_RR)),
           "v_xor_b32 v%d, v%d, v%d" % (S0, r(0), S0),
           "buffer_store_dword v%d, %%[voff], s[20:23], 0 offen" % S0,
           "s_add_u32 s20, s20, %[pitch]\n\ts_addc_u32 s21, s21, 0"]
    pending = []

    def flush(upto_all=False):
        while pending and (upto_all or len(pending) > XOR_DELAY):
            j = pending.pop(0)
            out.append("v_xor_b32 v%d, v%d, v%d" % (r(j), r(j), FBC))

    def update(i):
        if i == 0:
            cr = CRA if CRA % 4 not in (FBC % 4, r(0) % 4) else CRB
            out.append("v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (r(0), FBC, cr, r(0), IMM_R))
            return
        cr = CRA if CRA % 4 not in (r(i - 1) % 4, r(i) % 4) else CRB
        out.append("v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (r(i), r(i - 1), cr, r(i), IMM_R))
        if i in tapset:
            pending.append(i)
        flush()

    for i in range(N - 1, CTL_SR - 1, -1):
        update(i)
    flush(True)
    out.append("ds_write_b32 %%[xaddr], v%d offset:%d" % (r(CTL_SR), OFF_R53 + 256 * ph))
    out.append("s_waitcnt lgkmcnt(0)\n\ts_barrier")
    out.append("ds_read_b32 v%d, %%[xaddr] offset:%d" % (S54, OFF_S54 + 256 * ph))
    out.append("ds_read_b32 v%d, %%[xaddr] offset:%d" % (S0, OFF_S0 + 256 * ph))
    for i in range(CTL_SR - 1, -1, -1):
        update(i)
    flush(True)
    return out


# ------------------------------------------------------------------------- S wave
SR0 = 8                        # s_i home: v(SR0 + i)
G0, G1, CSR, R53, T159, SPARE = 2, 3, 4, 5, 6, 7
CTL_SS, CTL_RS = 106, 54       # c_S = s_106 ^ r_53; the R wave's control bit needs s_54
LAT = 8
LDS_LAT = 24
TA, TB, TC = 0xF0, 0xCC, 0xAA


class Op:
    __slots__ = ("kind", "text", "dst", "srcs")

    def __init__(self, kind, text, dst, srcs):
        self.kind, self.text, self.dst, self.srcs = kind, text, dst, list(srcs)


def s_body(tab):
    """Regions (split at the two barriers) of the S wave's two-clock body."""
    regions = [[], [], []]
    ring = [SR0 + i for i in range(N)]

    def emit(reg, kind, text, dst, srcs):
        regions[reg].append(Op(kind, text, dst, srcs))

    def v3(reg, dst, a, b, c, imm):
        emit(reg, "valu", "v_bitop3_b32 v%d, v%d, v%d, v%d bitop3:0x%02x" % (dst, a, b, c, imm), dst, (a, b, c))

    def v2(reg, name, dst, a, b):
        emit(reg, "valu", "%s v%d, v%d, v%d" % (name, dst, a, b), dst, (a, b))

    def sel(i, fbs):
        f0, f1 = i in tab["kFb0"], i in tab["kFb1"]
        return fbs if (f0 and f1) else G0 if f0 else G1 if f1 else None

    def update(reg, i, a, b, c, dst, fbs):
        bb = (TB ^ 0xFF) if i in tab["kComp0"] else TB
        cc = (TC ^ 0xFF) if i in tab["kComp1"] else TC
        v3(reg, dst, a, b, c, (TA ^ (bb & cc)) & 0xFF)
        if sel(i, fbs) is not None:
            v2(reg, "v_xor_b32", dst, dst, sel(i, fbs))

    assert sel(N - 1, 0) is not None, "the s_159 update is one op"
    for t in (0, 1):
        ph = 1 - t                      # clock t writes exchange parity (t + 1) & 1
        pre, post = t, t + 1
        fbs = ring[N - 1]
        v2(pre, "v_xor_b32", CSR, ring[CTL_SS], R53)
        v2(pre, "v_and_b32", G1, fbs, CSR)
        v2(pre, "v_xor_b32", G0, fbs, G1)
        new54 = None
        if t == 0:  # ascending: new s_i where old s_{i-1} was
            for i in range(1, N - 1):
                reg = pre if i <= CTL_RS else post
                update(reg, i, ring[i - 1], ring[i], ring[i + 1], ring[i - 1], fbs)
                if i == CTL_RS:
                    new54 = ring[i - 1]
            v2(post, "v_xor_b32", ring[N - 2], ring[N - 2], sel(N - 1, fbs))
            exports_after = None
            new_ring = [ring[N - 1]] + ring[:N - 1]
        else:  # descending: new s_159, s_158 in temporaries, new s_i where old s_{i+1} was
            t158 = CSR                  # c_S is dead once g1 and g0 are formed
            v2(pre, "v_xor_b32", T159, ring[N - 2], sel(N - 1, fbs))
            update(pre, N - 2, ring[N - 3], ring[N - 2], ring[N - 1], t158, fbs)
            for i in range(N - 3, 0, -1):
                reg = pre if i >= CTL_RS else post
                update(reg, i, ring[i - 1], ring[i], ring[i + 1], ring[i + 1], fbs)
                if i == CTL_RS:
                    new54 = ring[i + 1]
            new_ring = [ring[N - 1]] + ring[2:N - 1] + [t158, T159]
        # exchange: the new s_54 and the next s_0 (the old s_159), then the next r_53
        emit(pre, "ldsw", "ds_write_b32 %%[xaddr], v%d offset:%d" % (new54, OFF_S54 + 256 * ph), None, (new54,))
        emit(pre, "ldsw", "ds_write_b32 %%[xaddr], v%d offset:%d" % (fbs, OFF_S0 + 256 * ph), None, (fbs,))
        emit(pre, "barrier", "s_waitcnt lgkmcnt(0)\n\ts_barrier", None, ())
        emit(post, "ldsr", "ds_read_b32 v%d, %%[xaddr] offset:%d" % (R53, OFF_R53 + 256 * ph), R53, ())
        ring = new_ring
    # every word back to its home register (a parallel move; a cycle goes through SPARE)
    home = [SR0 + i for i in range(N)]
    pending = {home[i]: ring[i] for i in range(N) if ring[i] != home[i]}
    while pending:
        srcs = set(pending.values())
        ready = [d for d in pending if d not in srcs]
        if not ready:
            d = next(iter(pending))
            emit(2, "valu", "v_mov_b32 v%d, v%d" % (SPARE, pending[d]), SPARE, (pending[d],))
            pending[d] = SPARE
            continue
        for d in ready:
            emit(2, "valu", "v_mov_b32 v%d, v%d" % (d, pending[d]), d, (pending[d],))
            del pending[d]
    emit(2, "wait", "s_waitcnt lgkmcnt(0)", None, ())
    return regions


def schedule(ops):
    """List-schedule one region under RAW (LAT after VALU, LDS_LAT after an LDS read), WAR
    and WAW orders on physical registers; LDS ops keep their order; the barrier or wait
    stays last; LDS writes and the values they write go first."""
    tail = [o for o in ops if o.kind in ("barrier", "wait")]
    ops = [o for o in ops if o.kind not in ("barrier", "wait")]
    n = len(ops)
    preds = [[] for _ in range(n)]
    last_w, reads, prev_lds = {}, {}, None
    for k, o in enumerate(ops):
        for src in o.srcs:
            if src in last_w:
                w = ops[last_w[src]].kind
                preds[k].append((last_w[src], LDS_LAT if w == "ldsr" else LAT if w == "valu" else 1))
        if o.dst is not None:
            for rd in reads.get(o.dst, []):
                preds[k].append((rd, 1))
            if o.dst in last_w:
                preds[k].append((last_w[o.dst], 1))
        if o.kind in ("ldsw", "ldsr"):
            if prev_lds is not None:
                preds[k].append((prev_lds, 1))
            prev_lds = k
        for src in o.srcs:
            reads.setdefault(src, []).append(k)
        if o.dst is not None:
            last_w[o.dst] = k
            reads[o.dst] = []
    succs = [[] for _ in range(n)]
    for k in range(n):
        for p, d in preds[k]:
            succs[p].append((k, d))
    height = [0] * n
    for k in range(n - 1, -1, -1):
        height[k] = max([height[x] + d for x, d in succs[k]] + [1000 if ops[k].kind == "ldsw" else 0])
    npred = [len(p) for p in preds]
    ready_at = [0] * n
    avail = [k for k in range(n) if npred[k] == 0]
    order, slot = [], 0
    while avail:
        cands = [k for k in avail if ready_at[k] <= slot] or avail
        k = max(cands, key=lambda j: (height[j], -j))
        avail.remove(k)
        order.append(k)
        for x, d in succs[k]:
            ready_at[x] = max(ready_at[x], slot + d)
            npred[x] -= 1
            if npred[x] == 0:
                avail.append(x)
        slot += 1
    assert len(order) == n
    out, pending = [], set()
    for k in order:
        o = ops[k]
        if pending & set(o.srcs) or (o.dst is not None and o.dst in pending):
            out.append("s_waitcnt lgkmcnt(0)")
            pending = set()
        out.append(o.text)
        if o.kind == "ldsr":
            pending.add(o.dst)
    return out + [o.text for o in tail]


def s_texts(tab):
    texts = []
    for rg in s_body(tab):
        texts += schedule(rg)
    return texts




def clashes(texts):
    bad = 0
    for t in texts:
        if t.startswith("v_bitop3"):
            regs = sorted({int(x) for x in re.findall(r"v(\d+)", t)[1:4]})
            banks = [v % 4 for v in regs]
            bad += len(banks) - len(set(banks))
    return bad


def render() -> str:
    tab = tables()
    out = ["// Generated by gen_m128_loop.py from the tables of mickey128_bitslice.h; do not edit."]
    texts = clock(tab["kRTaps"], 1) + clock(tab["kRTaps"], 0)
    nvalu = sum(1 for t in texts if t.startswith("v_"))
    body = "\n\t".join(t.replace("\n", "\n\t") for t in texts)
    out += ["// R wave, 2 clocks per iteration: %d VALU (%.1f per clock), %d bitop3 bank clashes."
            % (nvalu, nvalu / 2, clashes(texts)),
            "#define M128_R_LOOP_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t")]
    state = ['"+{v%d}"(R(%d))' % (r(i), i) for i in range(N)]
    state += ['"+{v%d}"(S54)' % S54, '"+{v%d}"(S0)' % S0]
    out.append("#define M128_R_LOOP_STATE(R, S54, S0) \\\n    %s" % ", \\\n    ".join(state))
    out.append("#define M128_R_LOOP_CLOBBERS %s" % ", ".join('"v%d"' % v for v in sorted((CRA, CRB, FBC))))
    texts = s_texts(tab)
    nvalu = sum(1 for t in texts if t.startswith("v_"))
    body = "\n\t".join(t.replace("\n", "\n\t") for t in texts)
    out += ["// S wave, 2 clocks per iteration: %d VALU (%.1f per clock), %d bitop3 bank clashes."
            % (nvalu, nvalu / 2, clashes(texts)),
            "#define M128_S_LOOP_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t")]
    state = ['"+{v%d}"(S(%d))' % (SR0 + i, i) for i in range(N)] + ['"+{v%d}"(R53)' % R53]
    out.append("#define M128_S_LOOP_STATE(S, R53) \\\n    %s" % ", \\\n    ".join(state))
    out.append("#define M128_S_LOOP_CLOBBERS %s" % ", ".join('"v%d"' % v for v in (G0, G1, CSR, T159, SPARE)))
    return "\n".join(out) + "\n"


def main():
    text = render()
    with open(OUT, "w") as f:
        f.write(text)
    for line in text.split("\n"):
        if line.startswith("// R wave") or line.startswith("// S wave"):
            print(line)


if __name__ == "__main__":
    main()
