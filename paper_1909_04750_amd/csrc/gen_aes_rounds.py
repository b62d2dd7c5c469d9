#!/usr/bin/env python3
"""Writes aes_rounds.inc: four middle rounds of bitsliced AES-128 (SubBytes, ShiftRows,
MixColumns, AddRoundKey; FIPS-197 Sec. 5.1) as one inline-assembly body whose VGPRs are
placed for gfx950's register banks (a v_bitop3_b32 whose sources include two different
registers of one bank issues at about half rate; gen_clock_loop.py has the measurements).

State: plane b (most significant bit first) of state byte k is one VGPR.  The S-box is the
fused circuit of aes_sbox.h (read from that file); MixColumns and AddRoundKey are the
formulas of mix_add in aes_kernels.hip, with the round-key bit as a wave-uniform mask of
0 or all ones in an SGPR.

No copies: output byte k of a round (the S-box of input byte src(k) = r + 4((c + r) % 4),
then MixColumns) is written to the registers that held input byte src(k), which its own
S-box has consumed.  The byte -> register map thus follows ShiftRows, whose fourth power is
the identity, so after four rounds every byte is back in its home registers.  Within a
byte, bit b sits at home offset OFFS[b]: the S-box's first layer meets u3, u6 and u7 in
one three-source op, so u7 is not at offset 7 (same bank as u3).

Round keys: the body loads the 64 bytes of its four round keys with one s_load_dwordx16
into s[36:51] (from the address operand %[rk]) and turns each key bit into its mask with
s_bfe_i32 (sign-extended one-bit field) right before the VALU op that adds it, cycling
through s[52:59].

Ops are list-scheduled over a sliding window (dependent VALU ops LAT slots apart where
the window allows), then registers are allocated in that order: each new value takes a
free VGPR in the bank that clashes least with the registers already given to the other
sources of the ops that will read it.  v0..v7 are left to the compiler.

Run from this directory: python3 gen_aes_rounds.py  (rewrites aes_rounds.inc).
"""
from __future__ import annotations

import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "aes_rounds.inc")

ROUNDS = 4
OFFS = [0, 1, 2, 3, 7, 5, 6, 4]           # home offset of bit b within a byte's 8 registers
HOME0 = 8                                  # byte k's registers: HOME0 + 8k + OFFS[b]
VREGS = list(range(8, 256))
KEY_SGPR0 = 36                             # s[36:51]: 16 key dwords (4 rounds)
MASK_SGPRS = list(range(52, 60))
LAT = 4
WINDOW = 48
XOR3 = 0x96


def src_byte(k):
    r, c = k % 4, k // 4
    return r + 4 * ((c + r) % 4)


def parse_sbox():
    """The non-final S-box of aes_sbox.h as [(dst, kind, srcs, imm)] with inputs u0..u7
    and outputs s0..s7."""
    text = open(os.path.join(HERE, "aes_sbox.h")).read()
    body = text[text.index("void sbox("):]
    ops = []

    def name(tok):
        tok = tok.strip()
        m = re.fullmatch(r"u\[(\d)\]", tok)
        return "u%s" % m.group(1) if m else tok

    def expr(dst, e):
        e = e.strip().rstrip(";").strip()
        m = re.fullmatch(r"op3<0x([0-9A-Fa-f]+)>\((.*)\)", e)
        if m:
            a, b, c = (name(x) for x in m.group(2).split(","))
            ops.append((dst, "op3", [a, b, c], int(m.group(1), 16)))
            return
        m = re.fullmatch(r"~\((\w+) \^ (\w+)\)", e)
        if m:
            ops.append((dst, "xnor", [name(m.group(1)), name(m.group(2))], None))
            return
        m = re.fullmatch(r"(\S+) ([\^&]) (\S+)", e)
        if m:
            ops.append((dst, "xor" if m.group(2) == "^" else "and", [name(m.group(1)), name(m.group(3))], None))
            return
        raise ValueError("cannot parse S-box expression: " + e)
    for line in body.split("\n"):
        line = line.strip()
        m = re.match(r"const uint32_t (\w+) = (.*);$", line)
        if m:
            expr(m.group(1), m.group(2))
            continue
        m = re.match(r"s\[(\d)\] = FINAL \? .* : (.*);$", line)
        if m:
            expr("s" + m.group(1), m.group(2))
            continue
        m = re.match(r"s\[(\d)\] = (op3<.*);$", line)
        if m:
            expr("s" + m.group(1), m.group(2))
    outs = {d for d, _, _, _ in ops if re.fullmatch(r"s\d", d)}
    assert outs == {"s%d" % b for b in range(8)}, outs
    return ops


class Op:
    __slots__ = ("kind", "dst", "srcs", "imm", "sgpr", "key")

    def __init__(self, kind, dst, srcs, imm=None, key=None):
        self.kind, self.dst, self.srcs, self.imm, self.key = kind, dst, list(srcs), imm, key
        self.sgpr = None


def build_ops():
    """Value names: ('in', k, b) the body's inputs; (round, tag, ...) intermediates;
    ('st', round, k, b) round outputs."""
    sbox = parse_sbox()
    ops = []
    cur = {(k, b): ("in", k, b) for k in range(16) for b in range(8)}
    for rnd in range(ROUNDS):
        out = {}
        nxt = {}
        for c in range(4):  # a column's four S-boxes, then its MixColumns
            for k in range(4 * c, 4 * c + 4):
                s = src_byte(k)
                env = {"u%d" % b: cur[(s, b)] for b in range(8)}
                for dst, kind, srcs, imm in sbox:
                    v = (rnd, "sb", k, dst)
                    ops.append(Op(kind, v, [env[x] for x in srcs], imm))
                    env[dst] = v
                for b in range(8):
                    out[(k, b)] = env["s%d" % b]
            u = {}
            for r in range(4):
                for b in range(8):
                    v = (rnd, "u", c, r, b)
                    ops.append(Op("xor", v, [out[(4 * c + r, b)], out[(4 * c + (r + 1) % 4, b)]]))
                    u[(r, b)] = v
            for r in range(4):
                k = 4 * c + r
                for b in range(8):
                    a1 = out[(4 * c + (r + 1) % 4, b)]
                    u0 = lambda bb: u[(r, bb)]
                    u2 = u[((r + 2) % 4, b)]
                    t = (rnd, "t", k, b)
                    o = ("st", rnd, k, b)
                    if b in (3, 4, 6):
                        ops.append(Op("op3", t, [u0(b + 1), u0(0), a1], XOR3))
                        ops.append(Op("op3k", o, [t, u2], XOR3, key=(rnd, k, b)))
                    else:
                        ops.append(Op("op3", t, [u0(0) if b == 7 else u0(b + 1), a1, u2], XOR3))
                        ops.append(Op("xork", o, [t], None, key=(rnd, k, b)))
                    nxt[(k, b)] = o
        cur = nxt
    return ops, cur


def schedule(ops):
    """Windowed list scheduling: among the first WINDOW unscheduled ops (program order),
    take the one that is ready earliest, then the one with the longest path to the end."""
    n = len(ops)
    producer = {}
    for i, o in enumerate(ops):
        producer[o.dst] = i
    preds = [[producer[s] for s in o.srcs if s in producer] for o in ops]
    succs = [[] for _ in range(n)]
    for i, p in enumerate(preds):
        for j in p:
            succs[j].append(i)
    height = [0] * n
    for i in range(n - 1, -1, -1):
        height[i] = 1 + max([height[j] for j in succs[i]] or [0])
    done_at = {}
    order = []
    pending = list(range(n))
    slot = 0
    while pending:
        window = pending[:WINDOW]
        ready = [i for i in window if all(j in done_at for j in preds[i])]
        best = min(ready, key=lambda i: (max([done_at[j] + LAT for j in preds[i]] + [0]) > slot, -height[i], i))
        order.append(best)
        done_at[best] = slot
        pending.remove(best)
        slot += 1
    return [ops[i] for i in order]


def allocate(ops):
    """Register of every value.  State values are fixed: input byte k in byte slot k (8
    registers, HOME0 + 8k + OFFS[b]); round r's output byte k in the slot that held round
    r's input byte src(k).  Other values take a free non-slot VGPR, bank chosen against the
    already-placed partners of their future three-source reads."""
    slot = {k: k for k in range(16)}          # byte -> slot, for the round being built
    fixed = {}
    for rnd in range(ROUNDS):
        slot = {k: slot[src_byte(k)] for k in range(16)}
        for k in range(16):
            for b in range(8):
                fixed[("st", rnd, k, b)] = HOME0 + 8 * slot[k] + OFFS[b]
    assert slot == {k: k for k in range(16)}, "ShiftRows^4 returns every byte to its slot"
    homes = {HOME0 + 8 * k + OFFS[b] for k in range(16) for b in range(8)}
    reg = {("in", k, b): HOME0 + 8 * k + OFFS[b] for k in range(16) for b in range(8)}
    last_use = {}
    readers = {}
    for i, o in enumerate(ops):
        for s in o.srcs:
            last_use[s] = i
            readers.setdefault(s, []).append(i)
    # a slot register between its byte's last read and the next state value written there
    # can hold a value that dies before that write
    refill = {}
    for i, o in enumerate(ops):
        if o.dst in fixed:
            refill.setdefault(fixed[o.dst], []).append(i)
    free = set(VREGS) - homes
    free_slots = set()
    for i, o in enumerate(ops):
        for s in set(o.srcs):
            if last_use[s] == i:
                (free_slots if reg[s] in homes else free).add(reg[s])
        d = o.dst
        if d in fixed:
            r = fixed[d]
            if r not in free_slots:
                raise RuntimeError("slot register v%d of %s still in use" % (r, d))
            free_slots.discard(r)
        else:
            score = {0: 0, 1: 0, 2: 0, 3: 0}
            for j in readers.get(d, []):
                q = ops[j]
                if q.kind not in ("op3", "op3k"):
                    continue
                for s in q.srcs:
                    if s != d and s in reg:
                        score[reg[s] % 4] += 1
            end = last_use.get(d, len(ops))
            borrow = [x for x in free_slots if min([j for j in refill.get(x, []) if j > i] or [len(ops) + 1]) > end]
            cands = [(score[x % 4], 0, x) for x in free] + [(score[x % 4], 1, x) for x in borrow]
            if not cands:
                raise RuntimeError("out of VGPRs at op %d" % i)
            r = min(cands)[2]
            if r in free:
                free.discard(r)
            else:
                free_slots.discard(r)
        reg[d] = r
    return reg


def render_ops(ops, reg):
    texts = []
    mask_i = 0
    for o in ops:
        v = lambda x: "v%d" % reg[x]
        if o.kind in ("op3k", "xork"):
            rnd, k, b = o.key
            dword = KEY_SGPR0 + 4 * rnd + k // 4
            bit = 8 * (k % 4) + 7 - b          # byte k = byte k%4 of dword k//4 (little-endian)
            sg = MASK_SGPRS[mask_i % len(MASK_SGPRS)]
            mask_i += 1
            texts.append("s_bfe_i32 s%d, s%d, 0x%x" % (sg, dword, bit | (1 << 16)))
            if o.kind == "op3k":
                texts.append("v_bitop3_b32 %s, %s, %s, s%d bitop3:0x%02x" % (v(o.dst), v(o.srcs[0]), v(o.srcs[1]), sg, o.imm))
            else:
                texts.append("v_xor_b32 %s, s%d, %s" % (v(o.dst), sg, v(o.srcs[0])))
        elif o.kind == "op3":
            texts.append("v_bitop3_b32 %s, %s, %s, %s bitop3:0x%02x" % (v(o.dst), v(o.srcs[0]), v(o.srcs[1]), v(o.srcs[2]), o.imm))
        elif o.kind == "xnor":
            texts.append("v_bitop3_b32 %s, %s, %s, %s bitop3:0xc3" % (v(o.dst), v(o.srcs[0]), v(o.srcs[1]), v(o.srcs[1])))
        elif o.kind in ("xor", "and"):
            texts.append("v_%s_b32 %s, %s, %s" % (o.kind, v(o.dst), v(o.srcs[0]), v(o.srcs[1])))
        else:
            raise ValueError(o.kind)
    return texts


def clashes(texts):
    bad = 0
    for t in texts:
        if t.startswith("v_bitop3"):
            regs = sorted({int(x) for x in re.findall(r"\bv(\d+)", t)[1:4]})
            banks = [r % 4 for r in regs]
            bad += len(banks) - len(set(banks))
    return bad


def render() -> str:
    ops, _ = build_ops()
    ops = schedule(ops)
    reg = allocate(ops)
    texts = ["s_load_dwordx16 s[%d:%d], %%[rk], 0x0" % (KEY_SGPR0, KEY_SGPR0 + 15), "s_waitcnt lgkmcnt(0)"]
    texts += render_ops(ops, reg)
    nvalu = sum(1 for t in texts if t.startswith("v_"))
    nsalu = sum(1 for t in texts if t.startswith("s_"))
    used = sorted(set(reg.values()))
    homes = {HOME0 + 8 * k + OFFS[b] for k in range(16) for b in range(8)}
    clob = [r for r in used if r not in homes]
    body = "\n\t".join(texts)
    out = ["// Generated by gen_aes_rounds.py from aes_sbox.h; do not edit.",
           "// %d rounds: %d VALU (%d per round), %d scalar, %d bitop3 bank clashes, VGPRs v%d..v%d."
           % (ROUNDS, nvalu, nvalu // ROUNDS, nsalu, clashes(texts), min(used), max(used)),
           "#define AES_ROUNDS_COUNT %d" % ROUNDS,
           "#define AES_ROUNDS_BODY \\\n    \"%s\\n\"" % body.replace("\n", "\\n\" \\\n    \"").replace("\t", "\\t")]
    state = ['"+{v%d}"(ST(%d, %d))' % (HOME0 + 8 * k + OFFS[b], k, b) for k in range(16) for b in range(8)]
    out.append("#define AES_ROUNDS_STATE(ST) \\\n    %s" % ", \\\n    ".join(state))
    out.append("#define AES_ROUNDS_CLOBBERS %s" % ", ".join(
        ['"v%d"' % r for r in clob] + ['"s%d"' % s for s in range(KEY_SGPR0, KEY_SGPR0 + 16)] +
        ['"s%d"' % s for s in MASK_SGPRS] + ['"scc"']))  # s_bfe_i32 writes SCC
    return "\n".join(out) + "\n"


def main():
    text = render()
    with open(OUT, "w") as f:
        f.write(text)
    print(text.split("\n")[1])


if __name__ == "__main__":
    main()
