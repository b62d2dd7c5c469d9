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

}  // namespace mickey
