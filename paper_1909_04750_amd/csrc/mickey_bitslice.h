// Bitsliced MICKEY 2.0 clock for gfx950.
//
// One lane holds K 32-bit words per register bit: bit l of word k is instance 32k+l of
// the lane's group.  The 100 R words and 100 S words stay in VGPRs across clocks; every
// update is written as explicit v_bitop3_b32 / v_xor_b32 so that the instruction count
// per clock is the algorithmic one:
//
//   c_R = s_34 ^ r_67, c_S = s_67 ^ r_33                       2
//   g1 = fb_S & c_S, g0 = fb_S ^ g1                             2
//   R (descending, in place): r_i <- r_{i-1} ^ (c_R & r_i)       100  (one bitop3 each)
//        ^ fb_R where i is a feedback tap (tap 0 folds in)       49
//   S (ascending): s_i <- s_{i-1} ^ ((s_i^C0_i) & (s_{i+1}^C1_i)) 98  (complements are
//        folded into the bitop3 truth table at compile time)
//        ^ g0 / g1 / fb_S where FB0_i / FB1_i select it       76  (s_0 is a rename)
//   z = r_0 ^ s_0                                                1
//                                                              ---
//                                                              328 per 32 instances
//
// Cipher structure (paper Sec. II-C-1; the specification it cites): R is a Galois LFSR
// whose clocking with control bit 1 also adds the old register into itself; S is the
// non-linear register with complement masks COMP0/COMP1 and control-selected feedback
// masks FB0/FB1; each register's control bit comes from the other register.
#pragma once
#include "bitmatrix.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace mickey {

// ---------------------------------------------------------------------------------
// Register tables of MICKEY 2.0, as sets of positions i (0..99) where the entry is 1.
// R feedback taps:
constexpr uint8_t kRTaps[] = {0,  1,  3,  4,  5,  6,  9,  12, 13, 16, 19, 20, 21, 22, 25, 28, 37,
                              38, 41, 42, 45, 46, 50, 52, 54, 56, 58, 60, 61, 63, 64, 65, 66, 67,
                              71, 72, 79, 80, 81, 82, 87, 88, 89, 90, 91, 92, 94, 95, 96, 97};
// S complement masks (defined for 1 <= i <= 98):
constexpr uint8_t kComp0[] = {4,  5,  9,  11, 12, 13, 14, 16, 19, 21, 23, 25, 27, 29, 30, 32, 35,
                              43, 45, 47, 49, 54, 56, 59, 60, 61, 62, 65, 67, 69, 70, 71, 72, 73,
                              74, 75, 76, 77, 79, 81, 82, 83, 84, 85, 86, 88, 90, 97, 98};
constexpr uint8_t kComp1[] = {1,  3,  4,  7,  9,  10, 11, 12, 15, 17, 21, 22, 24, 26, 27, 28, 30, 31,
                              32, 33, 37, 38, 40, 42, 43, 44, 49, 53, 55, 56, 57, 61, 62, 63, 64, 65,
                              66, 68, 70, 71, 72, 74, 75, 76, 77, 81, 86, 87, 88, 92, 95, 96};
// S feedback masks for control bit 0 and 1:
constexpr uint8_t kFb0[] = {0,  1,  2,  3,  5,  7,  8,  9,  10, 11, 12, 13, 14, 17, 19, 20, 21, 22,
                            23, 24, 25, 26, 27, 28, 31, 32, 39, 40, 41, 44, 47, 49, 51, 54, 56, 57,
                            58, 59, 61, 63, 65, 75, 76, 78, 82, 83, 85, 86, 87, 90, 91, 92, 95, 96};
constexpr uint8_t kFb1[] = {0,  1,  2,  4,  5,  6,  11, 12, 13, 15, 18, 19, 23, 26, 27, 30, 32, 33,
                            37, 38, 44, 45, 47, 48, 52, 56, 59, 62, 64, 65, 67, 69, 72, 74, 78, 79,
                            80, 81, 83, 84, 85, 86, 87, 94, 99};

template <size_t N>
constexpr bool in_set(const uint8_t (&set)[N], int i)
{
    for (size_t k = 0; k < N; k++)
        if (set[k] == i) return true;
    return false;
}

template <size_t N>
constexpr int set_size(const uint8_t (&)[N]) { return (int)N; }

using bitops::TA;
using bitops::TB;
using bitops::TC;

// Algorithmic VALU ops per clock per word (see the table at the top).
constexpr int ops_per_clock()
{
    int fb = 0;
    for (int i = 1; i < 100; i++) fb += (in_set(kFb0, i) || in_set(kFb1, i)) ? 1 : 0;
    return 2 + 2 + 100 + (set_size(kRTaps) - 1) + 98 + fb + 1;
}
static_assert(in_set(kRTaps, 0), "tap 0 is folded into the r_0 update");
static_assert(in_set(kFb0, 0) && in_set(kFb1, 0), "s_0 update is a rename of the feedback bit");
static_assert(ops_per_clock() == 328, "op count of the clock");

// ---------------------------------------------------------------------------------
// K-word slicing word (K = 1: 32 instances per lane; K = 2: 64 instances per lane).
template <int K>
struct Word {
    uint32_t w[K];
};

template <int IMM, int K>
__device__ __forceinline__ Word<K> b3(const Word<K> &a, const Word<K> &b, const Word<K> &c)
{
    Word<K> r;
#pragma unroll
    for (int k = 0; k < K; k++) r.w[k] = __builtin_amdgcn_bitop3_b32(a.w[k], b.w[k], c.w[k], IMM);
    return r;
}
template <int K>
__device__ __forceinline__ Word<K> operator^(const Word<K> &a, const Word<K> &b)
{
    Word<K> r;
#pragma unroll
    for (int k = 0; k < K; k++) r.w[k] = a.w[k] ^ b.w[k];
    return r;
}
template <int K>
__device__ __forceinline__ Word<K> operator&(const Word<K> &a, const Word<K> &b)
{
    Word<K> r;
#pragma unroll
    for (int k = 0; k < K; k++) r.w[k] = a.w[k] & b.w[k];
    return r;
}
template <int K>
__device__ __forceinline__ Word<K> wzero()
{
    Word<K> r;
#pragma unroll
    for (int k = 0; k < K; k++) r.w[k] = 0u;
    return r;
}

template <int K>
struct Regs {
    Word<K> r[100];
    Word<K> s[100];
};

// R update, position I (descending order keeps it in place: r_I is rewritten after
// r_{I+1} has consumed it).
template <int I, int K>
__device__ __forceinline__ void r_step(Regs<K> &x, const Word<K> &cr, const Word<K> &fbr)
{
    if constexpr (I == 0) {
        x.r[0] = b3<TA ^ (TB & TC)>(fbr, cr, x.r[0]);  // 0 + feedback (tap 0) + c_R & r_0
    } else {
        Word<K> v = b3<TA ^ (TB & TC)>(x.r[I - 1], cr, x.r[I]);
        if constexpr (in_set(kRTaps, I)) v = v ^ fbr;
        x.r[I] = v;
    }
}

template <int K, int... J>
__device__ __forceinline__ void r_all(Regs<K> &x, const Word<K> &cr, const Word<K> &fbr,
                                      std::integer_sequence<int, J...>)
{
    (r_step<99 - J, K>(x, cr, fbr), ...);
}

// S update at position I in 1..98 (ascending): `prev` carries the old s_{I-1}.
template <int I, int K, bool MASKED>
__device__ __forceinline__ void s_step(Regs<K> &x, Word<K> &prev, const Word<K> &fbs, const Word<K> &g0,
                                       const Word<K> &g1, const Word<K> &m)
{
    constexpr int bb = in_set(kComp0, I) ? (TB ^ 0xFF) : TB;
    constexpr int cc = in_set(kComp1, I) ? (TC ^ 0xFF) : TC;
    constexpr int imm = (TA ^ (bb & cc)) & 0xFF;
    Word<K> old = x.s[I];
    Word<K> v = b3<imm>(prev, x.s[I], x.s[I + 1]);
    constexpr bool f0 = in_set(kFb0, I), f1 = in_set(kFb1, I);
    if constexpr (f0 && f1) v = v ^ fbs;
    else if constexpr (f0) v = v ^ g0;
    else if constexpr (f1) v = v ^ g1;
    // Masked clocks (initialisation with lanes not started yet, whose registers are
    // zero and whose inputs are zero): the only positions where an all-zero register
    // would turn non-zero are those with COMP0_i = COMP1_i = 1; clear them for idle lanes.
    if constexpr (MASKED && in_set(kComp0, I) && in_set(kComp1, I)) v = v & m;
    x.s[I] = v;
    prev = old;
}

template <int K, bool MASKED, int... J>
__device__ __forceinline__ void s_all(Regs<K> &x, Word<K> &prev, const Word<K> &fbs, const Word<K> &g0,
                                      const Word<K> &g1, const Word<K> &m, std::integer_sequence<int, J...>)
{
    (s_step<J + 1, K, MASKED>(x, prev, fbs, g0, g1, m), ...);
}

// One CLOCK_KG given the two feedback bits (fb_R = r_99 ^ input_R, fb_S = s_99 ^ input_S)
// already formed from the pre-clock state.
template <int K, bool MASKED>
__device__ __forceinline__ void clock_core(Regs<K> &x, const Word<K> &fbr, const Word<K> &fbs, const Word<K> &m)
{
    const Word<K> cr = x.s[34] ^ x.r[67];
    const Word<K> cs = x.s[67] ^ x.r[33];
    const Word<K> g1 = fbs & cs;  // feedback into FB1 positions (control 1)
    const Word<K> g0 = fbs ^ g1;  // feedback into FB0 positions (control 0)
    r_all<K>(x, cr, fbr, std::make_integer_sequence<int, 100>{});
    Word<K> prev = x.s[0];
    s_all<K, MASKED>(x, prev, fbs, g0, g1, m, std::make_integer_sequence<int, 98>{});
    {  // s_99 <- old s_98, plus feedback where selected
        Word<K> v = prev;
        constexpr bool f0 = in_set(kFb0, 99), f1 = in_set(kFb1, 99);
        if constexpr (f0 && f1) v = v ^ fbs;
        else if constexpr (f0) v = v ^ g0;
        else if constexpr (f1) v = v ^ g1;
        x.s[99] = v;
    }
    x.s[0] = fbs;  // s_0 <- feedback (FB0_0 = FB1_0 = 1)
}

// Keystream clock: mixing off, input 0.
template <int K>
__device__ __forceinline__ void clock_gen(Regs<K> &x)
{
    const Word<K> fbr = x.r[99];
    const Word<K> fbs = x.s[99];
    clock_core<K, false>(x, fbr, fbs, fbr);
}

// ---------------------------------------------------------------------------------
// Next value of one register position as a function of the current state (nothing is
// overwritten): used where a clock is computed in an order other than the in-place
// sweeps above (the four-wave split computes the positions other waves need first).
template <int I, int K>
__device__ __forceinline__ Word<K> r_next(const Regs<K> &x, const Word<K> &cr, const Word<K> &fbr)
{
    if constexpr (I == 0) {
        return b3<TA ^ (TB & TC)>(fbr, cr, x.r[0]);
    } else {
        Word<K> v = b3<TA ^ (TB & TC)>(x.r[I - 1], cr, x.r[I]);
        if constexpr (in_set(kRTaps, I)) v = v ^ fbr;
        return v;
    }
}

template <int I, int K>
__device__ __forceinline__ Word<K> s_next(const Regs<K> &x, const Word<K> &fbs, const Word<K> &g0,
                                          const Word<K> &g1)
{
    if constexpr (I == 0) {
        return fbs;
    } else {
        Word<K> v;
        if constexpr (I == 99) {
            v = x.s[98];
        } else {
            constexpr int bb = in_set(kComp0, I) ? (TB ^ 0xFF) : TB;
            constexpr int cc = in_set(kComp1, I) ? (TC ^ 0xFF) : TC;
            constexpr int imm = (TA ^ (bb & cc)) & 0xFF;
            v = b3<imm>(x.s[I - 1], x.s[I], x.s[I + 1]);
        }
        constexpr bool f0 = in_set(kFb0, I), f1 = in_set(kFb1, I);
        if constexpr (f0 && f1) v = v ^ fbs;
        else if constexpr (f0) v = v ^ g0;
        else if constexpr (f1) v = v ^ g1;
        return v;
    }
}

// ---------------------------------------------------------------------------------
// Split keystream clock: one wave holds R, another holds S of the same instances, and
// the two control bits cross between them (c_R needs s_34, c_S needs r_33).  Each half
// is cut where the value the other wave needs for the next clock is final: R runs
// r_99..r_33 (r_33 of the next state is then known), S runs s_1..s_34.
constexpr int kRCut = 33, kSCut = 34;  // the taps of c_S = s_67 ^ r_33 and c_R = s_34 ^ r_67

template <int K, int J0, int... J>
__device__ __forceinline__ void r_range(Regs<K> &x, const Word<K> &cr, const Word<K> &fbr,
                                        std::integer_sequence<int, J...>)
{
    (r_step<99 - (J0 + J), K>(x, cr, fbr), ...);
}
// r_99 .. r_{kRCut}
template <int K>
__device__ __forceinline__ void r_upper(Regs<K> &x, const Word<K> &cr, const Word<K> &fbr)
{
    r_range<K, 0>(x, cr, fbr, std::make_integer_sequence<int, 100 - kRCut>{});
}
// r_{kRCut-1} .. r_0
template <int K>
__device__ __forceinline__ void r_lower(Regs<K> &x, const Word<K> &cr, const Word<K> &fbr)
{
    r_range<K, 100 - kRCut>(x, cr, fbr, std::make_integer_sequence<int, kRCut>{});
}

template <int K, int I0, int... J>
__device__ __forceinline__ void s_range(Regs<K> &x, Word<K> &prev, const Word<K> &fbs, const Word<K> &g0,
                                        const Word<K> &g1, std::integer_sequence<int, J...>)
{
    (s_step<I0 + J, K, false>(x, prev, fbs, g0, g1, fbs), ...);
}
// s_1 .. s_{kSCut}; prev must hold the old s_0 on entry
template <int K>
__device__ __forceinline__ void s_lower(Regs<K> &x, Word<K> &prev, const Word<K> &fbs, const Word<K> &g0,
                                        const Word<K> &g1)
{
    s_range<K, 1>(x, prev, fbs, g0, g1, std::make_integer_sequence<int, kSCut>{});
}
// s_{kSCut+1} .. s_98, then s_99 and s_0
template <int K>
__device__ __forceinline__ void s_upper(Regs<K> &x, Word<K> &prev, const Word<K> &fbs, const Word<K> &g0,
                                        const Word<K> &g1)
{
    s_range<K, kSCut + 1>(x, prev, fbs, g0, g1, std::make_integer_sequence<int, 98 - kSCut>{});
    Word<K> v = prev;
    constexpr bool f0 = in_set(kFb0, 99), f1 = in_set(kFb1, 99);
    if constexpr (f0 && f1) v = v ^ fbs;
    else if constexpr (f0) v = v ^ g0;
    else if constexpr (f1) v = v ^ g1;
    x.s[99] = v;
    x.s[0] = fbs;
}

// The same S update as a descending sweep, for the split S wave: `nxt` carries the old
// s_{I+1}.  An ascending sweep leaves the new s_i in the register of the old s_{i-1}
// (the value that dies at that step) and a descending one in that of the old s_{i+1},
// so alternating the two returns every word to its register every two clocks with one
// spare register and no copies (a wave holds one register set, not two).
template <int I, int K>
__device__ __forceinline__ void s_step_desc(Regs<K> &x, Word<K> &nxt, const Word<K> &fbs, const Word<K> &g0,
                                            const Word<K> &g1)
{
    constexpr int bb = in_set(kComp0, I) ? (TB ^ 0xFF) : TB;
    constexpr int cc = in_set(kComp1, I) ? (TC ^ 0xFF) : TC;
    constexpr int imm = (TA ^ (bb & cc)) & 0xFF;
    Word<K> old = x.s[I];
    Word<K> v = b3<imm>(x.s[I - 1], x.s[I], nxt);
    constexpr bool f0 = in_set(kFb0, I), f1 = in_set(kFb1, I);
    if constexpr (f0 && f1) v = v ^ fbs;
    else if constexpr (f0) v = v ^ g0;
    else if constexpr (f1) v = v ^ g1;
    x.s[I] = v;
    nxt = old;
}

template <int K, int HI, int... J>
__device__ __forceinline__ void s_range_desc(Regs<K> &x, Word<K> &nxt, const Word<K> &fbs, const Word<K> &g0,
                                             const Word<K> &g1, std::integer_sequence<int, J...>)
{
    (s_step_desc<HI - J, K>(x, nxt, fbs, g0, g1), ...);
}
// s_99 (from the old s_98), then s_98 .. s_{kSCut}; returns nothing, leaves the old
// s_{kSCut} in nxt
template <int K>
__device__ __forceinline__ void s_upper_desc(Regs<K> &x, Word<K> &nxt, const Word<K> &fbs, const Word<K> &g0,
                                             const Word<K> &g1)
{
    nxt = x.s[99];
    Word<K> v = x.s[98];
    constexpr bool f0 = in_set(kFb0, 99), f1 = in_set(kFb1, 99);
    if constexpr (f0 && f1) v = v ^ fbs;
    else if constexpr (f0) v = v ^ g0;
    else if constexpr (f1) v = v ^ g1;
    x.s[99] = v;
    s_range_desc<K, 98>(x, nxt, fbs, g0, g1, std::make_integer_sequence<int, 98 - kSCut + 1>{});
}
// s_{kSCut-1} .. s_1, then s_0
template <int K>
__device__ __forceinline__ void s_lower_desc(Regs<K> &x, Word<K> &nxt, const Word<K> &fbs, const Word<K> &g0,
                                             const Word<K> &g1)
{
    s_range_desc<K, kSCut - 1>(x, nxt, fbs, g0, g1, std::make_integer_sequence<int, kSCut - 1>{});
    x.s[0] = fbs;
}

// Initialisation clock: mixing on, input word `in` (one input bit per lane).
template <int K, bool MASKED>
__device__ __forceinline__ void clock_mix(Regs<K> &x, const Word<K> &in, const Word<K> &m)
{
    const Word<K> fbr = b3<TA ^ TB ^ TC>(x.r[99], in, x.s[50]);  // r_99 ^ (in ^ s_50)
    const Word<K> fbs = x.s[99] ^ in;
    clock_core<K, MASKED>(x, fbr, fbs, m);
}

}  // namespace mickey
