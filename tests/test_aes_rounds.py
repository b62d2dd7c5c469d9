"""CPU checks of the generated bitsliced AES rounds (paper_1909_04750_amd/csrc/aes_rounds.inc):

- the committed file is what gen_aes_rounds.py produces from aes_sbox.h;
- every register the body reads is a state register or was written before;
- run by a small register-level emulator (VGPRs over lanes, SGPRs, the scalar key load and
  bit-field extract), the body takes every instance (bit of a lane's words) through the
  same four rounds as a byte-oriented reference built from the oracle's S-box, GF(2^8)
  multiplication and key expansion (FIPS-197 Sec. 5.1: SubBytes, ShiftRows, MixColumns,
  AddRoundKey), for two different key offsets.
"""
import importlib.util
import os
import re

import numpy as np

from oracle import aes as aes_oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")
INC = os.path.join(CSRC, "aes_rounds.inc")


def generator():
    spec = importlib.util.spec_from_file_location("gen_aes_rounds", os.path.join(CSRC, "gen_aes_rounds.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def parse():
    text = open(INC).read()
    rounds = int(re.search(r"#define AES_ROUNDS_COUNT (\d+)", text).group(1))
    body = re.search(r"#define AES_ROUNDS_BODY \\\n(.*?)\n#define", text, re.S).group(1)
    insts = [s.replace("\\t", "").replace("\\n", "").strip() for s in re.findall(r'"(.*?)"', body)]
    insts = [i for i in insts if i]
    homes = {(int(k), int(b)): int(v) for v, k, b in re.findall(r'"\+\{v(\d+)\}"\(ST\((\d+), (\d+)\)\)', text)}
    return rounds, insts, homes


def test_committed_rounds_match_generator():
    assert generator().render() == open(INC).read()


def test_registers_written_before_read():
    _, insts, homes = parse()
    written = set(homes.values())
    for ins in insts:
        op, _, rest = ins.partition(" ")
        if not op.startswith("v_"):
            continue
        regs = [int(x) for x in re.findall(r"\bv(\d+)", rest)]
        assert all(r in written for r in regs[1:]), ins
        written.add(regs[0])


def emulate(insts, vregs, key_bytes):
    """Run the body; key_bytes: the 64 bytes at the body's key address."""
    sregs = {}
    for ins in insts:
        op, _, rest = ins.partition(" ")
        args = [a.strip() for a in rest.split(",")]
        if op == "s_load_dwordx16":
            lo, hi = (int(x) for x in re.match(r"s\[(\d+):(\d+)\]", args[0]).groups())
            words = np.frombuffer(bytes(key_bytes), dtype="<u4")
            assert hi - lo + 1 == 16 and len(words) == 16
            for i in range(16):
                sregs[lo + i] = int(words[i])
            continue
        if op == "s_waitcnt":
            continue
        if op == "s_bfe_i32":
            d, a = int(args[0][1:]), int(args[1][1:])
            field = int(args[2], 16)
            off, width = field & 31, (field >> 16) & 127
            assert width == 1
            sregs[d] = 0xFFFFFFFF if (sregs[a] >> off) & 1 else 0
            continue

        def val(tok):
            tok = tok.split()[0]
            if tok.startswith("v"):
                return vregs[int(tok[1:])]
            return np.uint32(sregs[int(tok[1:])])
        d = int(args[0][1:])
        if op == "v_bitop3_b32":
            va, vb, vc = val(args[1]), val(args[2]), val(args[3])
            imm = int(args[3].split("bitop3:")[1], 16)
            out = np.zeros_like(vregs[next(iter(vregs))])
            for m in range(8):
                if imm >> m & 1:
                    out |= (va if m & 4 else ~va) & (vb if m & 2 else ~vb) & (vc if m & 1 else ~vc)
            vregs[d] = out
        elif op == "v_xor_b32":
            vregs[d] = (val(args[1]) ^ val(args[2])).astype(np.uint32)
        elif op == "v_and_b32":
            vregs[d] = (val(args[1]) & val(args[2])).astype(np.uint32)
        else:
            raise AssertionError("unexpected instruction " + ins)


def reference_round(state, rk):
    """One middle round of FIPS-197 on a 16-byte state (byte k = row k%4, column k//4)."""
    sb = [aes_oracle.sbox(x) for x in state]
    sr = [sb[(k % 4) + 4 * (((k // 4) + (k % 4)) % 4)] for k in range(16)]
    out = []
    for c in range(4):
        a = sr[4 * c: 4 * c + 4]
        for r in range(4):
            out.append(aes_oracle.gmul(a[r], 2) ^ aes_oracle.gmul(a[(r + 1) % 4], 3) ^ a[(r + 2) % 4] ^ a[(r + 3) % 4])
    return [out[k] ^ rk[k] for k in range(16)]


def test_rounds_equal_reference():
    rounds, insts, homes = parse()
    rng = np.random.default_rng(197)
    lanes = 2
    key = bytes(rng.integers(0, 256, 16, dtype=np.uint8))
    ek = aes_oracle.expand_key(key)
    for first in (2, 6):  # the kernel runs rounds 2-5 and 6-9
        key_bytes = ek[16 * first: 16 * (first + rounds)]
        states = rng.integers(0, 256, (lanes, 32, 16), dtype=np.uint8)  # lane, bit of the word, byte
        vregs = {v: rng.integers(0, 2 ** 32, lanes, dtype=np.uint64).astype(np.uint32) for v in range(256)}
        for (k, b), v in homes.items():
            bits = (states[:, :, k] >> (7 - b)) & 1
            vregs[v] = (bits.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)
        emulate(insts, vregs, key_bytes)
        for lane in range(lanes):
            for j in (0, 7, 31):
                st = [int(x) for x in states[lane, j]]
                for rnd in range(rounds):
                    st = reference_round(st, ek[16 * (first + rnd): 16 * (first + rnd + 1)])
                got = [sum(((int(vregs[homes[(k, b)]][lane]) >> j) & 1) << (7 - b) for b in range(8)) for k in range(16)]
                assert got == st, (first, lane, j)
