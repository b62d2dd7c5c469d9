// Bitsliced MICKEY-128 2.0 clock for gfx950 (the 128-bit-key member of the MICKEY 2.0
// family named in paper Sec. II-C-1): two 160-bit registers, bitsliced as in Sec. IV-D
// with 32 instances per 32-bit word.
//
// A slice's 320 state words do not fit one wave's 256 VGPRs, so a workgroup of two
// waves serves 64 slices: wave 0 keeps the 160 R words, wave 1 the 160 S words, and the
// two swap the control-bit inputs (and, for the keystream bit, s_0) through LDS once per
// clock.  Per clock and per 32 instances:
//
//   c_R = s_54 ^ r_106, c_S = s_106 ^ r_53                     2
//   g1 = fb_S & c_S, g0 = fb_S ^ g1                              2
//   R: r_i <- r_{i-1} ^ (c_R & r_i), in place, descending         160 bitop3
//      ^ fb_R at the 78 feedback taps (tap 0 folds in)             77
//   S: s_i <- s_{i-1} ^ ((s_i^C0_i) & (s_{i+1}^C1_i)), i=1..158    158 bitop3
//      ^ g0 / g1 / fb_S where FB0_i / FB1_i select it             118 (s_0 is a rename)
//   z = r_0 ^ s_0                                                 1
//                                                                ---
//                                                                518
//
// Tables.  The R taps are the cipher's (x^160 + sum x^i over the taps is primitive, and
// clocking with control bit 1 is multiplication by x + 1 = x^J, J = 2^80 - 255).  The
// four S tables are a stand-in (drawn once from splitmix64 with seed 0x128, keeping the
// 80-bit cipher's structure: complements unused at 0 and 159, FB0_0 = FB1_0 = 1); the
// kernels are table-driven, so the specification's S tables drop in as a table edit.
#pragma once
#include "bitmatrix.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace mickey128 {

constexpr int kN = 160;  // register length

// R feedback taps.
constexpr uint8_t kRTaps[] = {0,   4,   5,   8,   10,  11,  14,  16,  20,  25,  30,  32,  35,  36,  38,  42,
                              43,  46,  50,  51,  53,  54,  55,  56,  57,  60,  61,  62,  63,  65,  66,  69,
                              73,  74,  76,  79,  80,  81,  82,  85,  86,  90,  91,  92,  95,  97,  100, 101,
                              105, 106, 107, 108, 109, 111, 112, 113, 115, 116, 117, 127, 128, 129, 130, 131,
                              133, 135, 136, 137, 140, 142, 145, 148, 150, 152, 153, 154, 156, 157};
// S complement masks (used for 1 <= i <= 158), as sets of positions holding 1.
constexpr uint8_t kComp0[] = {1,   3,   5,   6,   7,   9,   10,  11,  12,  17,  21,  23,  24,  27,  28,  30,
                              31,  32,  33,  35,  38,  40,  41,  42,  43,  44,  45,  48,  49,  51,  55,  60,
                              61,  62,  64,  65,  66,  67,  70,  72,  75,  76,  78,  79,  81,  82,  83,  89,
                              90,  94,  97,  102, 103, 104, 106, 108, 111, 112, 113, 115, 116, 117, 121, 125,
                              129, 135, 137, 138, 139, 141, 144, 145, 149, 150, 151, 152, 153, 154, 158};
constexpr uint8_t kComp1[] = {2,   7,   8,   15,  16,  25,  27,  29,  30,  34,  36,  37,  40,  42,  44,  47,
                              48,  49,  53,  55,  59,  60,  61,  62,  63,  64,  65,  69,  72,  73,  75,  78,
                              79,  81,  82,  83,  87,  88,  89,  91,  95,  96,  100, 102, 107, 111, 112, 116,
                              118, 120, 121, 122, 123, 124, 126, 133, 135, 139, 140, 142, 144, 147, 150, 152,
                              155, 157, 158};
// S feedback masks for control bit 0 and 1.
constexpr uint8_t kFb0[] = {0,   1,   4,   5,   6,   11,  16,  19,  20,  22,  23,  24,  25,  30,  31,  32,
                            34,  39,  42,  43,  45,  46,  48,  50,  51,  54,  56,  59,  61,  63,  64,  66,
                            68,  70,  71,  73,  75,  76,  77,  78,  79,  82,  86,  88,  95,  97,  101, 105,
                            108, 112, 113, 118, 119, 120, 122, 123, 125, 126, 129, 131, 134, 137, 145, 147,
                            150, 153, 154, 155, 156, 158, 159};
constexpr uint8_t kFb1[] = {0,   2,   3,   6,   7,   9,   12,  15,  16,  17,  19,  24,  25,  28,  31,  33,
                            36,  37,  38,  39,  43,  46,  48,  49,  50,  54,  55,  56,  59,  60,  62,  63,
                            66,  67,  69,  70,  72,  73,  74,  76,  78,  79,  80,  81,  82,  83,  84,  86,
                            87,  89,  90,  91,  92,  94,  95,  98,  102, 103, 108, 109, 110, 111, 112, 113,
                            114, 117, 118, 122, 125, 126, 127, 133, 135, 136, 137, 140, 141, 142, 143, 144,
                            150, 154, 157, 158};

// Control and mixing taps.
constexpr int kCtlRS = 54, kCtlRR = 106;  // c_R = s_54 ^ r_106
constexpr int kCtlSS = 106, kCtlSR = 53;  // c_S = s_106 ^ r_53
constexpr int kMixS = 80;                 // with mixing on, s_80 enters R's feedback

template <size_t N>
constexpr bool in_set(const uint8_t (&set)[N], int i)
{
    for (size_t k = 0; k < N; k++)
        if (set[k] == i) return true;
    return false;
}

constexpr int ops_per_clock()
{
    int fb = 0;
    for (int i = 1; i < kN; i++) fb += (in_set(kFb0, i) || in_set(kFb1, i)) ? 1 : 0;
    return 2 + 2 + kN + ((int)sizeof(kRTaps) - 1) + (kN - 2) + fb + 1;
}
static_assert(sizeof(kRTaps) == 78 && in_set(kRTaps, 0), "78 taps, tap 0 folded into the r_0 update");
static_assert(in_set(kFb0, 0) && in_set(kFb1, 0), "s_0 update is a rename of the feedback bit");
static_assert(ops_per_clock() == 518, "op count of the clock");

using bitops::TA;
using bitops::TB;
using bitops::TC;

template <int IMM>
__device__ __forceinline__ uint32_t b3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
}

struct RRegs {
    uint32_t r[kN];
};
struct SRegs {
    uint32_t s[kN];
};

// ------------------------------------------------------------------------ R wave
// Position I of the R update; descending order keeps it in place.
template <int I>
__device__ __forceinline__ void r_step(RRegs &x, uint32_t cr, uint32_t fbr)
{
    if constexpr (I == 0) {
        x.r[0] = b3<TA ^ (TB & TC)>(fbr, cr, x.r[0]);
    } else {
        uint32_t v = b3<TA ^ (TB & TC)>(x.r[I - 1], cr, x.r[I]);
        if constexpr (in_set(kRTaps, I)) v ^= fbr;
        x.r[I] = v;
    }
}

template <int HI, int... J>
__device__ __forceinline__ void r_seq(RRegs &x, uint32_t cr, uint32_t fbr, std::integer_sequence<int, J...>)
{
    (r_step<HI - J>(x, cr, fbr), ...);
}
// r_HI down to r_LO
template <int HI, int LO>
__device__ __forceinline__ void r_range(RRegs &x, uint32_t cr, uint32_t fbr)
{
    r_seq<HI>(x, cr, fbr, std::make_integer_sequence<int, HI - LO + 1>{});
}

// ------------------------------------------------------------------------ S wave
// The selected feedback added to position I's update.
template <int I>
__device__ __forceinline__ uint32_t s_feedback(uint32_t v, uint32_t fbs, uint32_t g0, uint32_t g1)
{
    constexpr bool f0 = in_set(kFb0, I), f1 = in_set(kFb1, I);
    if constexpr (f0 && f1) return v ^ fbs;
    else if constexpr (f0) return v ^ g0;
    else if constexpr (f1) return v ^ g1;
    else return v;
}

// Position I in 1..158 (ascending); `prev` carries the old s_{I-1}.  With MASKED, lanes
// whose mask bit is 0 (not started yet: all-zero registers and input) stay zero: on a
// zero register only the positions with C0_I = C1_I = 1 would turn non-zero.
template <int I, bool MASKED>
__device__ __forceinline__ void s_step(SRegs &x, uint32_t &prev, uint32_t fbs, uint32_t g0, uint32_t g1, uint32_t m)
{
    constexpr int bb = in_set(kComp0, I) ? (TB ^ 0xFF) : TB;
    constexpr int cc = in_set(kComp1, I) ? (TC ^ 0xFF) : TC;
    constexpr int imm = (TA ^ (bb & cc)) & 0xFF;
    const uint32_t old = x.s[I];
    uint32_t v = s_feedback<I>(b3<imm>(prev, x.s[I], x.s[I + 1]), fbs, g0, g1);
    if constexpr (MASKED && in_set(kComp0, I) && in_set(kComp1, I)) v &= m;
    x.s[I] = v;
    prev = old;
}

template <int LO, bool MASKED, int... J>
__device__ __forceinline__ void s_seq(SRegs &x, uint32_t &prev, uint32_t fbs, uint32_t g0, uint32_t g1, uint32_t m,
                                      std::integer_sequence<int, J...>)
{
    (s_step<LO + J, MASKED>(x, prev, fbs, g0, g1, m), ...);
}
// s_LO up to s_HI (1 <= LO <= HI <= 158)
template <int LO, int HI, bool MASKED>
__device__ __forceinline__ void s_range(SRegs &x, uint32_t &prev, uint32_t fbs, uint32_t g0, uint32_t g1, uint32_t m)
{
    s_seq<LO, MASKED>(x, prev, fbs, g0, g1, m, std::make_integer_sequence<int, HI - LO + 1>{});
}
// s_159 <- old s_158 (in prev) plus the selected feedback; s_0 <- fb_S
__device__ __forceinline__ void s_top(SRegs &x, uint32_t prev, uint32_t fbs, uint32_t g0, uint32_t g1)
{
    x.s[kN - 1] = s_feedback<kN - 1>(prev, fbs, g0, g1);
    x.s[0] = fbs;
}

// The same update as a descending sweep: `nxt` carries the old s_{I+1}.  An ascending
// sweep leaves new s_i where old s_{i-1} was (the value that dies at that step), a
// descending one where old s_{i+1} was, so a clock of each returns every word to its
// register with one spare and no copies; the loops below alternate them.
template <int I, bool MASKED>
__device__ __forceinline__ void s_step_desc(SRegs &x, uint32_t &nxt, uint32_t fbs, uint32_t g0, uint32_t g1,
                                            uint32_t m)
{
    constexpr int bb = in_set(kComp0, I) ? (TB ^ 0xFF) : TB;
    constexpr int cc = in_set(kComp1, I) ? (TC ^ 0xFF) : TC;
    constexpr int imm = (TA ^ (bb & cc)) & 0xFF;
    const uint32_t old = x.s[I];
    uint32_t v = s_feedback<I>(b3<imm>(x.s[I - 1], x.s[I], nxt), fbs, g0, g1);
    if constexpr (MASKED && in_set(kComp0, I) && in_set(kComp1, I)) v &= m;
    x.s[I] = v;
    nxt = old;
}

template <int HI, bool MASKED, int... J>
__device__ __forceinline__ void s_seq_desc(SRegs &x, uint32_t &nxt, uint32_t fbs, uint32_t g0, uint32_t g1,
                                           uint32_t m, std::integer_sequence<int, J...>)
{
    (s_step_desc<HI - J, MASKED>(x, nxt, fbs, g0, g1, m), ...);
}
// s_HI down to s_LO (1 <= LO <= HI <= 158)
template <int HI, int LO, bool MASKED>
__device__ __forceinline__ void s_range_desc(SRegs &x, uint32_t &nxt, uint32_t fbs, uint32_t g0, uint32_t g1,
                                             uint32_t m)
{
    s_seq_desc<HI, MASKED>(x, nxt, fbs, g0, g1, m, std::make_integer_sequence<int, HI - LO + 1>{});
}
// First step of a descending sweep: returns the old s_159 and writes the new one.
__device__ __forceinline__ uint32_t s_top_desc(SRegs &x, uint32_t fbs, uint32_t g0, uint32_t g1)
{
    const uint32_t old = x.s[kN - 1];
    x.s[kN - 1] = s_feedback<kN - 1>(x.s[kN - 2], fbs, g0, g1);
    return old;
}

}  // namespace mickey128
