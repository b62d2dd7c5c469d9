"""CPU builds of the host-side C and C++ under AddressSanitizer and UndefinedBehaviorSanitizer.

- The oracles (oracle/*.c) are compiled into small drivers that run their known-answer
  vectors (tests/golden), every IV length, multi-instance generation with skips and the
  state packing; the drivers print the keystreams, which must equal the published
  vectors (for MICKEY-128 2.0, which has none here, the ordinary build's output).  Any
  out-of-bounds access or undefined operation aborts the driver.
- The serving allocator (csrc/arena.h) runs the random alloc/release sequences of
  tests/test_arena.py.
Host code only: nothing here touches a GPU.
"""
import os
import subprocess

import pytest

from tests import test_arena

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
GOLDEN = os.path.join(ROOT, "tests", "golden")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

MICKEY_DRIVER = r"""
#include "mickey_ref.c"
#include <stdio.h>
#include <stdlib.h>
static void hex(const uint8_t *p, size_t n) { for (size_t i = 0; i < n; i++) printf("%02x", p[i]); printf("\n"); }
static int unhex(const char *s, uint8_t *out) { int n = 0; for (; s[0] && s[1]; s += 2) { unsigned v; sscanf(s, "%2x", &v); out[n++] = (uint8_t)v; } return n; }
int main(int argc, char **argv)
{
    /* argv: key iv iv_bits nbytes, repeated */
    for (int a = 1; a + 3 < argc; a += 4) {
        uint8_t key[10] = {0}, iv[10] = {0}, out[64];
        unhex(argv[a], key);
        unhex(argv[a + 1], iv);
        mref_state st;
        if (mref_init(&st, key, iv, (unsigned)atoi(argv[a + 2])) != 0) return 2;
        int nb = atoi(argv[a + 3]);
        mref_generate(&st, 8u * (uint64_t)nb, out);
        hex(out, (size_t)nb);
    }
    /* every IV length, several instances with a skip, pack/unpack, a rejected length */
    uint8_t keys[81 * 10], ivs[81 * 10], lens[81], rows[81 * 13];
    for (int i = 0; i < 81 * 10; i++) { keys[i] = (uint8_t)(i * 37 + 11); ivs[i] = (uint8_t)(i * 91 + 5); }
    for (int i = 0; i < 81; i++) lens[i] = (uint8_t)i;
    if (mref_generate_many(keys, ivs, lens, 81, 17, 100, rows) != 0) return 3;
    mref_state st;
    uint8_t packed[25];
    mref_init(&st, keys, ivs, 80);
    mref_pack_state(&st, packed);
    mref_unpack_state(&st, packed);
    lens[3] = 81;
    if (mref_generate_many(keys, ivs, lens, 81, 0, 8, rows) != -1) return 4;
    return 0;
}
"""

GRAIN_DRIVER = r"""
#include "grain_ref.c"
#include <stdio.h>
static void hex(const uint8_t *p, size_t n) { for (size_t i = 0; i < n; i++) printf("%02x", p[i]); printf("\n"); }
static void unhex(const char *s, uint8_t *out) { int n = 0; for (; s[0] && s[1]; s += 2) { unsigned v; sscanf(s, "%2x", &v); out[n++] = (uint8_t)v; } }
int main(int argc, char **argv)
{
    for (int a = 1; a + 1 < argc; a += 2) {
        uint8_t key[10], iv[8], out[10];
        unhex(argv[a], key);
        unhex(argv[a + 1], iv);
        gref_state st;
        gref_init(&st, key, iv);
        gref_generate(&st, 80, out);
        hex(out, 10);
    }
    uint8_t keys[50], ivs[40], rows[5 * 9], packed[20];
    for (int i = 0; i < 50; i++) keys[i] = (uint8_t)(i * 29 + 3);
    for (int i = 0; i < 40; i++) ivs[i] = (uint8_t)(i * 53 + 1);
    gref_generate_many(keys, ivs, 5, 33, 72, rows);
    gref_state st;
    gref_init(&st, keys, ivs);
    gref_pack_state(&st, packed);
    gref_unpack_state(&st, packed);
    return 0;
}
"""

AES_DRIVER = r"""
#include "aes_ref.c"
#include <stdio.h>
static void hex(const uint8_t *p, size_t n) { for (size_t i = 0; i < n; i++) printf("%02x", p[i]); printf("\n"); }
static void unhex(const char *s, uint8_t *out) { int n = 0; for (; s[0] && s[1]; s += 2) { unsigned v; sscanf(s, "%2x", &v); out[n++] = (uint8_t)v; } }
int main(int argc, char **argv)
{
    for (int a = 1; a + 1 < argc; a += 2) {
        uint8_t key[16], in[16], out[16];
        unhex(argv[a], key);
        unhex(argv[a + 1], in);
        aref_encrypt(key, in, out);
        hex(out, 16);
    }
    uint8_t key[16], ctr[3 * 16], out[3 * 2 * 16];
    for (int i = 0; i < 16; i++) key[i] = (uint8_t)i;
    for (int i = 0; i < 48; i++) ctr[i] = (uint8_t)(0xF0 + i);
    aref_ctr_many(key, ctr, 3, 5, 2, out);
    for (int a = 0; a < 256; a++) (void)aref_sbox((uint8_t)a);
    return 0;
}
"""


MICKEY128_DRIVER = r"""
#include "mickey128_ref.c"
#include <stdio.h>
static void hex(const uint8_t *p, size_t n) { for (size_t i = 0; i < n; i++) printf("%02x", p[i]); printf("\n"); }
int main(void)
{
    /* every IV length 0..128 with a skip, the packed state, a rejected length */
    static uint8_t keys[129 * 16], ivs[129 * 16], lens[129], rows[129 * 13];
    for (int i = 0; i < 129 * 16; i++) { keys[i] = (uint8_t)(i * 37 + 11); ivs[i] = (uint8_t)(i * 91 + 5); }
    for (int i = 0; i < 129; i++) lens[i] = (uint8_t)i;
    if (m128_generate_many(keys, ivs, lens, 129, 17, 100, rows) != 0) return 3;
    for (int i = 0; i < 129; i += 32) hex(rows + 13 * i, 13);
    m128_state st;
    uint8_t packed[40];
    m128_init(&st, keys, ivs, 128);
    m128_pack_state(&st, packed);
    hex(packed, 40);
    lens[3] = 129;
    if (m128_generate_many(keys, ivs, lens, 129, 0, 8, rows) != -1) return 4;
    return 0;
}
"""


def golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(dict(kv.split("=", 1) for kv in line.split()[1 if line.startswith(("block", "ctr")) else 0:]))
    return rows


def build_and_run(tmp_path, name, driver, lang, args):
    src = tmp_path / ("%s.%s" % (name, lang))
    src.write_text(driver)
    exe = tmp_path / name
    cc = "gcc" if lang == "c" else "g++"
    std = "-std=c11" if lang == "c" else "-std=c++17"
    subprocess.check_call([cc, std, *SAN, "-I", ORACLE, "-I", os.path.join(ROOT, "paper_1909_04750_amd", "csrc"),
                           str(src), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe), *args], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    return res.stdout.split()


def test_mickey_oracle_under_sanitizers(tmp_path):
    kats = golden("mickey2_kat.txt")
    args = []
    for k in kats:
        args += [k["key"], k["iv"] or "00", k["iv_bits"], str(len(k["ks"]) // 2)]
    out = build_and_run(tmp_path, "mickey_san", MICKEY_DRIVER, "c", args)
    assert out == [k["ks"] for k in kats]


def test_grain_oracle_under_sanitizers(tmp_path):
    kats = golden("grain_v1_kat.txt")
    args = []
    for k in kats:
        args += [k["key"], k["iv"]]
    out = build_and_run(tmp_path, "grain_san", GRAIN_DRIVER, "c", args)
    assert out == [k["ks"] for k in kats]


def test_aes_oracle_under_sanitizers(tmp_path):
    blocks = [r for r in golden("aes128_kat.txt") if "in" in r]
    args = []
    for b in blocks:
        args += [b["key"], b["in"]]
    out = build_and_run(tmp_path, "aes_san", AES_DRIVER, "c", args)
    assert out == [b["out"] for b in blocks]


def test_mickey128_oracle_under_sanitizers(tmp_path):
    import numpy as np

    from oracle import mickey128 as m128
    out = build_and_run(tmp_path, "mickey128_san", MICKEY128_DRIVER, "c", [])
    i = np.arange(129 * 16)
    keys = ((i * 37 + 11) % 256).astype(np.uint8).reshape(129, 16)
    ivs = ((i * 91 + 5) % 256).astype(np.uint8).reshape(129, 16)
    rows = m128.generate_many(keys, ivs, np.arange(129, dtype=np.uint8), 100, skip=17)
    st = m128.State()
    st.init(keys[0].tobytes(), ivs[0].tobytes(), 128)
    assert out == [rows[k].tobytes().hex() for k in range(0, 129, 32)] + [st.packed().hex()]


def test_arena_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "arena_san", test_arena.HARNESS, "cpp", [])
    assert out and out[0] == "ok"
