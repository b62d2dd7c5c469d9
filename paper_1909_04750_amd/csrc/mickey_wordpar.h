// Word-parallel MICKEY 2.0 clock for latency mode: one instance per lane, each 100-bit
// register held as four 32-bit words (bit i of the register is bit i%32 of word i/32;
// bits 100..127 of word 3 are don't-care).  A clock costs ~50 VALU ops for one instance
// (the bitsliced clock costs 328 ops for 32 instances), but a lone instance advances
// ~6x faster, which is what the longest requests of a batch need (paper Sec. VI names
// delay as the main drawback of GPU generators).
//
// The masks below are derived at compile time from the same position sets as the
// bitsliced clock (mickey_bitslice.h), so the two representations share one table.
#pragma once
#include "mickey_bitslice.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mickey {

template <size_t N>
constexpr uint32_t set_word(const uint8_t (&set)[N], int k)
{
    uint32_t w = 0;
    for (size_t j = 0; j < N; j++)
        if (set[j] / 32 == k) w |= 1u << (set[j] % 32);
    return w;
}

struct WordMasks {
    uint32_t taps[4], comp0[4], comp1[4], fb0[4], fb1[4], inner[4];  // inner: positions 1..98
};

constexpr WordMasks make_word_masks()
{
    WordMasks m{};
    for (int k = 0; k < 4; k++) {
        m.taps[k] = set_word(kRTaps, k);
        m.comp0[k] = set_word(kComp0, k);
        m.comp1[k] = set_word(kComp1, k);
        m.fb0[k] = set_word(kFb0, k);
        m.fb1[k] = set_word(kFb1, k);
        uint32_t in = 0;
        for (int b = 0; b < 32; b++) {
            const int i = 32 * k + b;
            if (i >= 1 && i <= 98) in |= 1u << b;
        }
        m.inner[k] = in;
    }
    return m;
}

constexpr WordMasks kWM = make_word_masks();

struct WState {
    uint32_t r[4], s[4];
};

// bit b of x as an all-zeros / all-ones mask
__device__ __forceinline__ uint32_t bitmask(uint32_t x, int b) { return (uint32_t)((int32_t)(x << (31 - b)) >> 31); }

// (hi:lo) >> s, low 32 bits
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, int s) { return __builtin_amdgcn_alignbit(hi, lo, s); }

// One CLOCK_KG.  in_m: input bit as a mask; MIX: mixing on (s_50 added to R's input).
template <bool MIX>
__device__ __forceinline__ void wclock(WState &x, uint32_t in_m)
{
    const uint32_t cr = bitmask(x.s[1], 34 - 32) ^ bitmask(x.r[2], 67 - 64);
    const uint32_t cs = bitmask(x.s[2], 67 - 64) ^ bitmask(x.r[1], 33 - 32);
    uint32_t fbr = bitmask(x.r[3], 99 - 96);
    if (MIX) fbr ^= in_m ^ bitmask(x.s[1], 50 - 32);
    const uint32_t fbs = bitmask(x.s[3], 99 - 96) ^ in_m;
    // R: shift up by one, feedback into the taps, plus the old register when cr
    const uint32_t rl0 = x.r[0] << 1, rl1 = funnel(x.r[1], x.r[0], 31), rl2 = funnel(x.r[2], x.r[1], 31),
                   rl3 = funnel(x.r[3], x.r[2], 31);
    const uint32_t rl[4] = {rl0, rl1, rl2, rl3};
    // S: s-hat_i = s_{i-1} ^ ((s_i ^ COMP0_i) & (s_{i+1} ^ COMP1_i)) on 1..98, s-hat_99 = s_98
    const uint32_t sl0 = x.s[0] << 1, sl1 = funnel(x.s[1], x.s[0], 31), sl2 = funnel(x.s[2], x.s[1], 31),
                   sl3 = funnel(x.s[3], x.s[2], 31);
    const uint32_t sr0 = funnel(x.s[1], x.s[0], 1), sr1 = funnel(x.s[2], x.s[1], 1), sr2 = funnel(x.s[3], x.s[2], 1),
                   sr3 = x.s[3] >> 1;
    const uint32_t sl[4] = {sl0, sl1, sl2, sl3}, sr[4] = {sr0, sr1, sr2, sr3};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t t = __builtin_amdgcn_bitop3_b32(rl[k], fbr, kWM.taps[k], TA ^ (TB & TC));  // rl ^ (fb & taps)
        x.r[k] = __builtin_amdgcn_bitop3_b32(t, cr, x.r[k], TA ^ (TB & TC));                      // ^ (cr & r)
        const uint32_t q = __builtin_amdgcn_bitop3_b32(x.s[k], kWM.comp0[k], kWM.inner[k], (TA ^ TB) & TC);
        const uint32_t y = sr[k] ^ kWM.comp1[k];
        const uint32_t h = __builtin_amdgcn_bitop3_b32(sl[k], q, y, TA ^ (TB & TC));              // sl ^ (q & y)
        const uint32_t fsel = __builtin_amdgcn_bitop3_b32(cs, kWM.fb1[k], kWM.fb0[k], (TA & TB) | (~TA & TC));
        x.s[k] = __builtin_amdgcn_bitop3_b32(h, fbs, fsel, TA ^ (TB & TC));                       // ^ (fbs & fsel)
    }
}

// ---------------------------------------------------------------------------------
// The same clock on four lanes (a quad) per instance: lane q keeps word q of R and of S.
// Per clock the quad XOR-reduces each lane's share of the four bits that steer the clock
// (s_34 ^ r_67 = c_R, r_33 ^ s_67 = c_S, r_99 = fb_R, s_99 = fb_S) with two DPP swaps,
// fetches its neighbours' words for the shifts with DPP quad permutes, and updates its two
// words: ~25 VALU per clock instead of ~52, i.e. about twice as fast for one instance (one
// wave issues at most ~0.4 instructions/ns, so the count per clock sets the speed).
// The shift up takes word q-1 from lane q-1 and, in lane 0, word 3 by a rotating permute:
// bits 100..127 of word 3 are kept zero often enough that the bit it shifts into r_0 and
// s_0 (bit 127) is always zero.  Those bits only ever take bit 99 shifted upwards (no tap,
// comparison or feedback position lies above 99), one position per clock, so clearing them
// every 16 clocks keeps bits 116..127 zero; quad_word does that.
// Every lane of a quad must be active.

constexpr int qp(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t bitmask_i(uint32_t v, int b) { return (uint32_t)((int32_t)(v << (31 - b)) >> 31); }

struct QuadMasks {
    uint32_t taps, comp0, comp1, fb0, fb1, inner;  // word q of the position masks
    uint32_t keep;                                 // lane 3: bits 96..99 only
    uint32_t ra, rm, sa, sm;                       // this lane's share of the steering bits
};

__device__ __forceinline__ uint32_t pick4(uint32_t q, uint32_t a, uint32_t b, uint32_t c, uint32_t d)
{
    return q == 0 ? a : q == 1 ? b : q == 2 ? c : d;
}

__device__ __forceinline__ QuadMasks quad_masks(uint32_t q)
{
    QuadMasks m;
    m.taps = pick4(q, kWM.taps[0], kWM.taps[1], kWM.taps[2], kWM.taps[3]);
    m.comp0 = pick4(q, kWM.comp0[0], kWM.comp0[1], kWM.comp0[2], kWM.comp0[3]);
    m.comp1 = pick4(q, kWM.comp1[0], kWM.comp1[1], kWM.comp1[2], kWM.comp1[3]);
    m.fb0 = pick4(q, kWM.fb0[0], kWM.fb0[1], kWM.fb0[2], kWM.fb0[3]);
    m.fb1 = pick4(q, kWM.fb1[0], kWM.fb1[1], kWM.fb1[2], kWM.fb1[3]);
    m.inner = pick4(q, kWM.inner[0], kWM.inner[1], kWM.inner[2], kWM.inner[3]);
    m.keep = q == 3 ? 0xFu : 0xFFFFFFFFu;
    // v bit 0: c_R (s_34 in lane 1, r_67 in lane 2), bit 1: c_S (r_33 in lane 1, s_67 in
    // lane 2), bit 2: fb_R (r_99, lane 3), bit 3: fb_S (s_99, lane 3)
    m.ra = pick4(q, 0, 0, 3, 1);
    m.rm = pick4(q, 0, 2, 1, 4);
    m.sa = pick4(q, 0, 2, 2, 0);
    m.sm = pick4(q, 0, 1, 2, 8);
    return m;
}

// One clock; bit 127 of r and s (word 3, bit 31) must be zero (see quad_word).
__device__ __forceinline__ void quad_clock(uint32_t &r, uint32_t &s, const QuadMasks &m)
{
    uint32_t v = ((r >> m.ra) & m.rm) ^ ((s >> m.sa) & m.sm);
    v ^= qperm<qp(1, 0, 3, 2)>(v);
    v ^= qperm<qp(2, 3, 0, 1)>(v);
    const uint32_t cr = bitmask_i(v, 0), cs = bitmask_i(v, 1), fbr = bitmask_i(v, 2), fbs = bitmask_i(v, 3);
    const uint32_t rp = qperm<qp(3, 0, 1, 2)>(r);  // lane 0: word 3, whose bit 31 is zero
    const uint32_t sp = qperm<qp(3, 0, 1, 2)>(s);
    const uint32_t sn = qperm<qp(1, 2, 3, 3)>(s);
    const uint32_t rl = __builtin_amdgcn_alignbit(r, rp, 31);  // register shifted up by one
    const uint32_t sl = __builtin_amdgcn_alignbit(s, sp, 31);
    const uint32_t sr = __builtin_amdgcn_alignbit(sn, s, 1);   // shifted down by one
    const uint32_t t = __builtin_amdgcn_bitop3_b32(rl, fbr, m.taps, TA ^ (TB & TC));
    r = __builtin_amdgcn_bitop3_b32(t, cr, r, TA ^ (TB & TC));
    const uint32_t qv = __builtin_amdgcn_bitop3_b32(s, m.comp0, m.inner, (TA ^ TB) & TC);
    const uint32_t y = sr ^ m.comp1;
    const uint32_t h = __builtin_amdgcn_bitop3_b32(sl, qv, y, TA ^ (TB & TC));
    const uint32_t fsel = __builtin_amdgcn_bitop3_b32(cs, m.fb1, m.fb0, (TA & TB) | (~TA & TC));
    s = __builtin_amdgcn_bitop3_b32(h, fbs, fsel, TA ^ (TB & TC));
}

// 32 clocks; returns their keystream bits, the first in the MSB (valid in lane 0).  Clears
// bits 100..127 before clocks 0 and 16, so any value of them on entry is allowed.
__device__ __forceinline__ uint32_t quad_word(uint32_t &r, uint32_t &s, const QuadMasks &m)
{
    uint32_t acc = 0;
#pragma unroll
    for (int b = 0; b < 32; b++) {
        if (b % 16 == 0) {
            r &= m.keep;
            s &= m.keep;
        }
        acc = __builtin_amdgcn_alignbit(r ^ s, acc, 1);  // z = r_0 ^ s_0 (lane 0) enters at bit 31
        quad_clock(r, s, m);
    }
    return __builtin_bitreverse32(acc);
}

}  // namespace mickey
