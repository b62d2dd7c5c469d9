// Bitsliced Grain (version 1) clock for gfx950.
//
// One lane holds one 32-bit word per register bit: bit l of every word belongs to
// instance l of the lane's slice.  The 80 NFSR words b and 80 LFSR words s stay in VGPRs.
// A shift register needs no data movement when bitsliced: the window is a ring of 80
// registers, and after clock t the oldest bit b_{t+1} sits in slot (t+1) % 80.  With the
// clock loop unrolled 80 times every slot index is a compile-time constant, so a clock is
// only its feedback and output arithmetic:
//
//   z   = b1^b2^b4^b10^b31^b43^b56 ^ h(s3, s25, s46, s64, b63)        9 ops
//         with h = A ^ (x2 & B), A = x1 ^ f(x0,x3,x4),
//         f = x4 ^ x0x3 ^ x3x4, B = (x3 & ~(x0^x4)) ^ MAJ(x0,x1,x4)
//   s80 = s0^s13^s23^s38^s51^s62                                         3 ops
//   b80 = s0 ^ g(b): 12 linear terms and 11 monomials, the monomials
//         built from 5 shared pair products                             24 ops
//                                                                       --
//                                                                       36 per 32 instances
// (in the 160 initialisation clocks z is also added to s80 and b80; the xor chains absorb
// it at the same op count).
//
// Cipher structure: the paper's Grain subsection (Sec. II-C) and the specification it
// cites (LFSR feedback polynomial, NFSR feedback g, filter h, output taps A).
#pragma once
#include "bitmatrix.h"

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace grain {

using bitops::TA;
using bitops::TB;
using bitops::TC;

constexpr int kXor3 = TA ^ TB ^ TC;
constexpr int kAnd3 = TA & TB & TC;
constexpr int kXorAnd = TA ^ (TB & TC);  // a ^ (b & c)
constexpr int kNot(int t) { return t ^ 0xFF; }
// filter pieces, operands named as in the table above
constexpr int kF = TC ^ (TA & TB) ^ (TB & TC);             // (x0, x3, x4): x4 ^ x0x3 ^ x3x4
constexpr int kMaj = (TA & TB) | (TA & TC) | (TB & TC);    // (x0, x1, x4)
constexpr int kB = (TA & kNot(TB)) ^ TC;                   // (x3, x0^x4, maj)

// Truth-table check of the filter decomposition against h's algebraic normal form.
constexpr int tt(int imm, int a, int b, int c) { return (imm >> ((a << 2) | (b << 1) | c)) & 1; }
constexpr bool filter_ok()
{
    for (int v = 0; v < 32; v++) {
        const int x0 = v & 1, x1 = v >> 1 & 1, x2 = v >> 2 & 1, x3 = v >> 3 & 1, x4 = v >> 4 & 1;
        const int h = x1 ^ x4 ^ (x0 & x3) ^ (x2 & x3) ^ (x3 & x4) ^ (x0 & x1 & x2) ^ (x0 & x2 & x3) ^
                      (x0 & x2 & x4) ^ (x1 & x2 & x4) ^ (x2 & x3 & x4);
        const int f = tt(kF, x0, x3, x4), mj = tt(kMaj, x0, x1, x4), bb = tt(kB, x3, x0 ^ x4, mj);
        if (tt(kXorAnd, x1 ^ f, x2, bb) != h) return false;
    }
    return true;
}
static_assert(filter_ok(), "h = A ^ (x2 & B)");

template <int IMM>
__device__ __forceinline__ uint32_t op3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, IMM);
}

constexpr int kRing = 80;
constexpr int kInitClocks = 160;
constexpr int ops_per_clock() { return 9 + 3 + 24; }

struct State {
    uint32_t b[kRing];  // NFSR window: b_{t+i} in slot (t + i) % 80
    uint32_t s[kRing];  // LFSR window
};

// Ring slot of register bit i when the oldest bit is in slot R.
constexpr int at(int R, int i) { return (R + i) % kRing; }

struct Next {
    uint32_t z, s80, b80;
};

// Output bit and both feedback bits of the window whose oldest bit is in slot R.  With
// INIT, z is added to both feedbacks (the initialisation clocks).
template <int R, bool INIT>
__device__ __forceinline__ Next step(const State &x)
{
    const uint32_t *b = x.b, *s = x.s;
#define GB(i) b[at(R, i)]
#define GS(i) s[at(R, i)]
    // z = sum_A b_k ^ h(s3, s25, s46, s64, b63)
    const uint32_t x0 = GS(3), x1 = GS(25), x2 = GS(46), x3 = GS(64), x4 = GB(63);
    const uint32_t f = op3<kF>(x0, x3, x4);
    const uint32_t m = x0 ^ x4;
    const uint32_t mj = op3<kMaj>(x0, x1, x4);
    const uint32_t bb = op3<kB>(x3, m, mj);
    // the sums are balanced trees of three-input XORs: one clock's work is a few short
    // chains rather than one long one, which two waves per SIMD could not hide
    const uint32_t a = op3<kXor3>(op3<kXor3>(GB(1), GB(2), GB(4)), op3<kXor3>(GB(10), GB(31), GB(43)),
                                  op3<kXor3>(GB(56), x1, f));
    const uint32_t z = op3<kXorAnd>(a, x2, bb);
    // s_{t+80}
    const uint32_t f1 = op3<kXor3>(GS(0), GS(13), GS(23)), f2 = op3<kXor3>(GS(38), GS(51), GS(62));
    const uint32_t fs = INIT ? op3<kXor3>(f1, f2, z) : (f1 ^ f2);
    // b_{t+80} = s_t ^ g(b): pair products shared by several monomials
    const uint32_t p1 = GB(63) & GB(60), p2 = GB(37) & GB(33), p3 = GB(15) & GB(9);
    const uint32_t p4 = GB(52) & GB(45), p5 = GB(28) & GB(21);
    const uint32_t m5 = GB(33) & p5;                       // b33 b28 b21
    const uint32_t t6 = op3<kAnd3>(GB(63), GB(45), GB(28));
    const uint32_t m7 = op3<kAnd3>(GB(60), GB(52), p2);    // b60 b52 b37 b33
    const uint32_t m8 = op3<kAnd3>(p1, GB(21), GB(15));    // b63 b60 b21 b15
    const uint32_t m9 = op3<kAnd3>(p1, p4, GB(37));        // b63 b60 b52 b45 b37
    const uint32_t m11 = op3<kAnd3>(p4, p2, p5);           // b52 b45 b37 b33 b28 b21
    const uint32_t g1 = op3<kXor3>(GS(0), GB(62), GB(60)), g2 = op3<kXor3>(GB(52), GB(45), GB(37));
    const uint32_t g3 = op3<kXor3>(GB(33), GB(28), GB(21)), g4 = op3<kXor3>(GB(14), GB(9), GB(0));
    const uint32_t g5 = op3<kXor3>(p1, p2, p3);             // b63 b60, b37 b33, b15 b9
    const uint32_t g6 = op3<kXor3>(m5, m7, m8);
    const uint32_t g7 = INIT ? op3<kXor3>(m9, m11, z) : (m9 ^ m11);
    const uint32_t q1 = op3<kXorAnd>(op3<kXor3>(g1, g2, g3), GB(60), p4);  // b60 b52 b45
    const uint32_t q2 = op3<kXorAnd>(op3<kXor3>(g4, g5, g6), t6, GB(9));   // b63 b45 b28 b9
    const uint32_t q3 = op3<kXorAnd>(g7, m5, p3);                          // b33 b28 b21 b15 b9
    const uint32_t g = op3<kXor3>(q1, q2, q3);
#undef GB
#undef GS
    return Next{z, fs, g};
}

// One clock in the ring: the new bits replace the oldest ones, in slot R.
template <int R, bool INIT>
__device__ __forceinline__ uint32_t clock_ring(State &x)
{
    const Next n = step<R, INIT>(x);
    x.s[R] = n.s80;
    x.b[R] = n.b80;
    return n.z;
}

// One clock with the oldest bit in slot 0 that moves every word down one slot, so the
// window stays in canonical order (for clock counts that are not a multiple of 80).
__device__ __forceinline__ uint32_t clock_shift(State &x)
{
    const Next n = step<0, false>(x);
#pragma unroll
    for (int i = 0; i < kRing - 1; i++) {
        x.s[i] = x.s[i + 1];
        x.b[i] = x.b[i + 1];
    }
    x.s[kRing - 1] = n.s80;
    x.b[kRing - 1] = n.b80;
    return n.z;
}

// 80 clocks starting and ending with the window in canonical order; z of clock R goes to
// emit(R, z).
template <bool INIT, class Emit, int... R>
__device__ __forceinline__ void ring80(State &x, Emit &&emit, std::integer_sequence<int, R...>)
{
    ((emit(R, clock_ring<R, INIT>(x))), ...);
}

template <bool INIT, class Emit>
__device__ __forceinline__ void clocks80(State &x, Emit &&emit)
{
    ring80<INIT>(x, emit, std::make_integer_sequence<int, kRing>{});
}

// The first n (< 80, wave-uniform) clocks of a revolution from canonical order: afterwards
// b_j and s_j sit in slot (j + n) % 80.
template <class Emit, int... R>
__device__ __forceinline__ void ring_prefix(State &x, uint32_t n, Emit &&emit, std::integer_sequence<int, R...>)
{
    ((R < (int)n ? (void)emit(R, clock_ring<R, false>(x)) : (void)0), ...);
}

}  // namespace grain
