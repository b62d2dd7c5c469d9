// Clock pairs of the four-wave split (the exchange schedule of s4_clock_* in mickey_device.h,
// paper Sec. IV-D's per-instance clock, bitsliced) run by the generated loop of
// mickey_split4_loop.inc: the same clocks and LDS slots, with the VGPRs fixed so that no
// fused op reads two registers of one bank.  Wave 0 also stores the keystream word of
// every clock (one bit-plane row, `pitch` bytes apart) through a buffer resource built in
// s[20:23] from `plane`; the other roles leave `plane` unused.
#pragma once

#include "mickey_device.h"
#include "mickey_split4_loop.inc"

namespace mickey {

// `iters` clock pairs (the first clock of each writes exchange buffer 1, the second
// buffer 0), starting from the registers and imports the s4_clock_* code holds after an
// exchange; at return they hold the state `2 * iters` clocks later.  iters == 0 is a no-op.
template <int ROLE>
__device__ __forceinline__ void s4_pairs(Regs<1> &x, S4In &in, Split4Lds &xl, uint32_t lane, const char *plane,
                                         uint32_t voff, uint32_t pitch32, uint32_t iters)
{
    if (iters == 0) return;
    const uint32_t xaddr = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)&xl.v[0][0][lane];
    const uint64_t base = (uint64_t)(uintptr_t)plane;
#define MICKEY_S4_ASM(BODY, STATE, CLOBBERS)                                                                      \
    asm volatile("s_mov_b32 s20, %[lo]\n\ts_and_b32 s21, %[hi], 0xffff\n\ts_mov_b32 s22, 0x7fffffff\n\t"          \
                 "s_mov_b32 s23, 0x20000\n\ts_mov_b32 s24, %[it]\n1:\n\t" BODY                                      \
                 "\n\ts_sub_u32 s24, s24, 1\n\ts_cmp_lg_u32 s24, 0\n\ts_cbranch_scc1 1b"                                \
                 : STATE                                                                                          \
                 : [lo] "s"((uint32_t)base), [hi] "s"((uint32_t)(base >> 32)), [pitch] "s"(pitch32),             \
                   [it] "s"(iters), [voff] "v"(voff), [xaddr] "v"(xaddr)                                          \
                 : CLOBBERS, "s20", "s21", "s22", "s23", "s24", "scc", "memory")
    if constexpr (ROLE == 0) MICKEY_S4_ASM(MICKEY_S4_BODY_0, MICKEY_S4_STATE_0, MICKEY_S4_CLOBBERS_0);
    else if constexpr (ROLE == 1) MICKEY_S4_ASM(MICKEY_S4_BODY_1, MICKEY_S4_STATE_1, MICKEY_S4_CLOBBERS_1);
    else if constexpr (ROLE == 2) MICKEY_S4_ASM(MICKEY_S4_BODY_2, MICKEY_S4_STATE_2, MICKEY_S4_CLOBBERS_2);
    else MICKEY_S4_ASM(MICKEY_S4_BODY_3, MICKEY_S4_STATE_3, MICKEY_S4_CLOBBERS_3);
#undef MICKEY_S4_ASM
}

}  // namespace mickey
