"""CPU test of the serving output-budget allocator (csrc/arena.h, host C++): random
allocation and release sequences never hand out overlapping or out-of-range blocks, a
block is at least as large as asked and at most 12.5% larger (beyond 8 words), the free
count is exact, and after everything is released the whole budget can be allocated
again as one block (the merge recovers fragmented space)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04750_amd", "csrc")

HARNESS = r"""
#include "arena.h"
#include <cstdio>
#include <random>
#include <set>
int main()
{
    serve_arena::Arena a;
    const size_t cap = 1 << 20;
    a.reset(cap);
    std::mt19937_64 rng(1);
    std::map<size_t, size_t> live;  // off -> granted
    size_t used = 0;
    long fails = 0;
    for (int step = 0; step < 200000; step++) {
        const bool big = rng() % 50 == 0;
        if (live.empty() || rng() % 100 < 55) {
            const size_t w = 1 + (big ? rng() % 60000 : (rng() % 3 ? rng() % 3000 : rng() % 20));
            size_t off, g;
            if (!a.alloc(w, &off, &g)) { fails++; continue; }
            if (g < w || (w > 8 && g * 8 > w * 9 + 8)) { printf("BAD size %zu %zu\n", w, g); return 1; }
            if (off + g > cap) { printf("BAD range\n"); return 1; }
            auto it = live.upper_bound(off);
            if (it != live.end() && off + g > it->first) { printf("BAD overlap next\n"); return 1; }
            if (it != live.begin()) { auto p = std::prev(it); if (p->first + p->second > off) { printf("BAD overlap prev\n"); return 1; } }
            live[off] = g;
            used += g;
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            a.release(it->first, it->second);
            used -= it->second;
            live.erase(it);
        }
        if (a.free_words() != cap - used) { printf("BAD free %zu %zu\n", a.free_words(), cap - used); return 1; }
    }
    for (auto &kv : live) a.release(kv.first, kv.second);
    size_t off, g;
    if (!a.alloc(cap, &off, &g) || off != 0) { printf("BAD final\n"); return 1; }
    // small budget: four 128-word blocks come and go, then a 2-word block stays while a
    // 208-word class must still fit beside it
    serve_arena::Arena b;
    b.reset(256);
    size_t o[4], gg;
    for (int r = 0; r < 2; r++) {
        for (int i = 0; i < 2; i++) if (!b.alloc(128, &o[i], &gg)) { printf("BAD small 1\n"); return 1; }
        for (int i = 0; i < 2; i++) b.release(o[i], 128);
    }
    size_t a1, a2;
    if (!b.alloc(2, &a1, &gg) || !b.alloc(200, &a2, &gg) || gg != 208) { printf("BAD small 2\n"); return 1; }
    printf("ok fails=%ld\n", fails);
    return 0;
}
"""


def test_arena_random_sequences(tmp_path):
    src = tmp_path / "a.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "a"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout
