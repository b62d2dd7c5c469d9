"""Generate aes_sbox.h: the AES S-box as a bitsliced straight-line program of
v_bitop3_b32 operations.

The circuit is Boyar and Peralta's depth-16 AES S-box circuit ("A depth-16 circuit for
the AES S-box", 2012): a linear top layer of 27 XORs, a non-linear middle section over
GF(2^4) built from 32-odd AND gates, and a linear bottom layer, 128 two-input gates in
all.  It is restated below gate by gate.  This script fuses it for gfx950's
three-input v_bitop3_b32: a gate whose value is used once and whose operands, together
with its consumer's other operands, number at most three is folded into the consumer, and
each remaining node becomes one bitop3 with the truth table of its fused expression.

Run: python3 gen_aes_sbox.py > aes_sbox.h   (the output is committed; the library build
does not run this script).
"""
import sys

CIRCUIT = """
T1 = U0 + U3
T2 = U0 + U5
T3 = U0 + U6
T4 = U3 + U5
T5 = U4 + U6
T6 = T1 + T5
T7 = U1 + U2
T8 = U7 + T6
T9 = U7 + T7
T10 = T6 + T7
T11 = U1 + U5
T12 = U2 + U5
T13 = T3 + T4
T14 = T6 + T11
T15 = T5 + T11
T16 = T5 + T12
T17 = T9 + T16
T18 = U3 + U7
T19 = T7 + T18
T20 = T1 + T19
T21 = U6 + U7
T22 = T7 + T21
T23 = T2 + T22
T24 = T2 + T10
T25 = T20 + T17
T26 = T3 + T16
T27 = T1 + T12
M1 = T13 x T6
M2 = T23 x T8
M3 = T14 + M1
M4 = T19 x U7
M5 = M4 + M1
M6 = T3 x T16
M7 = T22 x T9
M8 = T26 + M6
M9 = T20 x T17
M10 = M9 + M6
M11 = T1 x T15
M12 = T4 x T27
M13 = M12 + M11
M14 = T2 x T10
M15 = M14 + M11
M16 = M3 + M2
M17 = M5 + T24
M18 = M8 + M7
M19 = M10 + M15
M20 = M16 + M13
M21 = M17 + M15
M22 = M18 + M13
M23 = M19 + T25
M24 = M22 + M23
M25 = M22 x M20
M26 = M21 + M25
M27 = M20 + M21
M28 = M23 + M25
M29 = M28 x M27
M30 = M26 x M24
M31 = M20 x M23
M32 = M27 x M31
M33 = M27 + M25
M34 = M21 x M22
M35 = M24 x M34
M36 = M24 + M25
M37 = M21 + M29
M38 = M32 + M33
M39 = M23 + M30
M40 = M35 + M36
M41 = M38 + M40
M42 = M37 + M39
M43 = M37 + M38
M44 = M39 + M40
M45 = M42 + M41
M46 = M44 x T6
M47 = M40 x T8
M48 = M39 x U7
M49 = M43 x T16
M50 = M38 x T9
M51 = M37 x T17
M52 = M42 x T15
M53 = M45 x T27
M54 = M41 x T10
M55 = M44 x T13
M56 = M40 x T23
M57 = M39 x T19
M58 = M43 x T3
M59 = M38 x T22
M60 = M37 x T20
M61 = M42 x T1
M62 = M45 x T4
M63 = M41 x T2
L0 = M61 + M62
L1 = M50 + M56
L2 = M46 + M48
L3 = M47 + M55
L4 = M54 + M58
L5 = M49 + M61
L6 = M62 + L5
L7 = M46 + L3
L8 = M51 + M59
L9 = M52 + M53
L10 = M53 + L4
L11 = M60 + L2
L12 = M48 + M51
L13 = M50 + L0
L14 = M52 + M61
L15 = M55 + L1
L16 = M56 + L0
L17 = M57 + L1
L18 = M58 + L8
L19 = M63 + L4
L20 = L0 + L1
L21 = L1 + L7
L22 = L3 + L12
L23 = L18 + L2
L24 = L15 + L9
L25 = L6 + L10
L26 = L7 + L9
L27 = L8 + L10
L28 = L11 + L14
L29 = L11 + L17
S0 = L6 + L24
S1 = L16 # L26
S2 = L19 # L28
S3 = L6 + L21
S4 = L20 + L22
S5 = L25 + L29
S6 = L13 # L27
S7 = L6 # L23
"""
# '+' is XOR, 'x' is AND, '#' is XNOR.  Inputs U0..U7 and outputs S0..S7 are the bits of
# a byte, most significant first.

TA, TB, TC = 0xF0, 0xCC, 0xAA
# truth tables (operand c unused) that have plain C forms
TWO_INPUT = {TA ^ TB: "%s ^ %s", (TA ^ TB) ^ 0xFF: "~(%s ^ %s)", TA & TB: "%s & %s"}


def parse():
    gates = []
    for line in CIRCUIT.strip().splitlines():
        d, _, x, op, y = line.split()
        gates.append((d, x, op, y))
    return gates


def evaluate(node, defs, env):
    if node in env:
        return env[node]
    x, op, y = defs[node]
    a, b = evaluate(x, defs, env), evaluate(y, defs, env)
    return a ^ b if op == "+" else (a & b if op == "x" else 1 ^ a ^ b)


def main():
    gates = parse()
    defs = {d: (x, op, y) for d, x, op, y in gates}
    order = [g[0] for g in gates]
    uses = {}
    for d, x, op, y in gates:
        for v in (x, y):
            uses[v] = uses.get(v, 0) + 1
    outputs = ["S%d" % i for i in range(8)]

    def leaves(n, mat):
        if n.startswith("U") or n in mat:
            return [n]
        x, _, y = defs[n]
        out = []
        for v in leaves(x, mat) + leaves(y, mat):
            if v not in out:
                out.append(v)
        return out

    mat = {n for n in order if n in outputs or uses.get(n, 0) != 1}
    changed = True
    while changed:
        changed = False
        for n in order:
            if n not in mat:
                continue
            x, _, y = defs[n]
            if len(set(leaves(x, mat)) | set(leaves(y, mat))) > 3:
                lx, ly = leaves(x, mat), leaves(y, mat)
                cands = [c for c in ((x, lx), (y, ly)) if not (c[0].startswith("U") or c[0] in mat)]
                c = max(cands, key=lambda t: len(t[1]))[0]
                mat.add(c)
                changed = True
    nodes = [n for n in order if n in mat]

    def cname(v):
        return "u[%s]" % v[1:] if v.startswith("U") else v.lower()

    lines = []
    for n in nodes:
        x, _, y = defs[n]
        ops = leaves(x, mat)
        for v in leaves(y, mat):
            if v not in ops:
                ops.append(v)
        tt = 0
        for idx in range(8):
            bits = [(idx >> 2) & 1, (idx >> 1) & 1, idx & 1]
            env = {ops[k]: bits[k] for k in range(len(ops))}
            sub = dict(defs)
            for m in mat:  # stop expansion at materialised nodes
                if m in env:
                    sub.pop(m, None)
            tt |= evaluate(n, {k: v for k, v in defs.items() if k not in env}, env) << idx
        args = [cname(v) for v in ops] + ["0u"] * (3 - len(ops))
        expr = "op3<0x%02X>(%s, %s, %s)" % (tt, *args)
        if len(ops) == 2 and tt in TWO_INPUT:  # plain two-operand forms (VOP2 encodings)
            expr = TWO_INPUT[tt] % (args[0], args[1])
        if n in outputs:
            i = int(n[1:])
            if len(ops) <= 2:
                # the final round adds round-key bit k[i]: a free third operand
                ttk = 0
                for idx in range(8):
                    c = idx & 1
                    ttk |= (((tt >> (idx & 6)) & 1) ^ c) << idx
                lines.append("    s[%d] = FINAL ? op3<0x%02X>(%s, %s, k[%d]) : %s;" % (i, ttk, args[0], args[1], i, expr))
            else:
                lines.append("    s[%d] = %s;" % (i, expr))
                lines.append("    if (FINAL) s[%d] ^= k[%d];" % (i, i))
        else:
            lines.append("    const uint32_t %s = %s;" % (cname(n), expr))
    nops = len(nodes)
    w = sys.stdout.write
    w("// Generated by gen_aes_sbox.py (Boyar-Peralta depth-16 AES S-box circuit, fused into\n")
    w("// three-input v_bitop3_b32 operations); do not edit.\n")
    w("#pragma once\n#include <hip/hip_runtime.h>\n#include <stdint.h>\n\nnamespace aesbs {\n\n")
    w("template <int IMM>\n__device__ __forceinline__ uint32_t op3(uint32_t a, uint32_t b, uint32_t c)\n{\n")
    w("    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);\n}\n\n")
    w("constexpr int kSboxOps = %d;  // bitop3 per S-box (one more per output with FINAL and three operands)\n\n" % nops)
    w("// u[0..7]: the input byte's bit-planes, most significant bit first; s[0..7]: S-box output\n")
    w("// planes.  With FINAL, round-key planes k[0..7] are added to the outputs.\n")
    w("template <bool FINAL>\n__device__ __forceinline__ void sbox(const uint32_t (&u)[8], uint32_t (&s)[8], const uint32_t (&k)[8])\n{\n")
    w("\n".join(lines) + "\n}\n\n}  // namespace aesbs\n")


if __name__ == "__main__":
    main()
