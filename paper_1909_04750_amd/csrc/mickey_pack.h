// Moving single instances between the bitsliced plane layout, the word-parallel quad
// layout and the packed 25-byte state (r_0..r_99 then s_0..s_99, most significant bit
// first: the layout of mickey_state_export), for kernels that resume stored states (the
// server's pool, the per-instance requests of mickey_generate_batch).
#pragma once
#include "mickey_bitslice.h"
#include "mickey_wordpar.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mickey {

// Replace bit l of state words J0..J1-1 (0..99: r_j, 100..199: s_{j-100}) with the
// packed state at src (25 bytes, r_0..r_99 then s_0..s_99, most significant bit first).
template <int J0 = 0, int J1 = 200>
__device__ __forceinline__ void gather_lane(Regs<1> &x, uint32_t l, const uint8_t *src)
{
    uint32_t w[7];
#pragma unroll
    for (int k = 0; k < 7; k++) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int byte = 4 * k + b;
            const bool used = byte < 25 && byte * 8 + 7 >= J0 && byte * 8 < J1;
            v = (v << 8) | (used ? (uint32_t)src[byte] : 0u);
        }
        w[k] = v;
    }
    const uint32_t m = 1u << l;
    constexpr int kSel = (TA & ~TB & 0xFF) | (TC & TB);  // b ? c : a
#pragma unroll
    for (int j = J0; j < J1; j++) {
        const uint32_t bit = 0u - ((w[j >> 5] >> (31 - (j & 31))) & 1u);
        Word<1> &dst = j < 100 ? x.r[j] : x.s[j - 100];
        dst.w[0] = __builtin_amdgcn_bitop3_b32(dst.w[0], m, bit, kSel);
    }
}

// Pack bit l of the 200 state words into 25 bytes at dst (MSB first).
__device__ __forceinline__ void write_back_lane(const Regs<1> &x, uint32_t l, uint8_t *dst)
{
    uint32_t w[7];
#pragma unroll
    for (int k = 0; k < 7; k++) w[k] = 0u;
#pragma unroll
    for (int j = 0; j < 200; j++) {
        const uint32_t v = j < 100 ? x.r[j].w[0] : x.s[j - 100].w[0];
        w[j >> 5] |= ((v >> l) & 1u) << (31 - (j & 31));
    }
#pragma unroll
    for (int b = 0; b < 25; b++) dst[b] = (uint8_t)(w[b >> 2] >> (24 - 8 * (b & 3)));
}

// Bits J0..J1-1 of write_back_lane (0..99: r_j, 100..199: s_{j-100}), for the split
// schedules where each wave holds part of the registers.  Bytes wholly inside the range
// are stored; a byte shared with another part (at most one at each end) is updated with
// two atomics on its aligned word that touch only this part's bits (the other waves and
// the neighbouring states own the rest).
template <int J0, int J1>
__device__ __forceinline__ void write_back_range(const Regs<1> &x, uint32_t l, uint8_t *dst)
{
    uint32_t w[7];
#pragma unroll
    for (int k = 0; k < 7; k++) w[k] = 0u;
#pragma unroll
    for (int j = J0; j < J1; j++) {
        const uint32_t v = j < 100 ? x.r[j].w[0] : x.s[j - 100].w[0];
        w[j >> 5] |= ((v >> l) & 1u) << (31 - (j & 31));
    }
#pragma unroll
    for (int b = J0 / 8; b < (J1 + 7) / 8; b++) {
        const uint32_t v = (w[b >> 2] >> (24 - 8 * (b & 3))) & 0xFFu;
        const int lo = 8 * b > J0 ? 8 * b : J0, hi = 8 * b + 8 < J1 ? 8 * b + 8 : J1;
        if (lo == 8 * b && hi == 8 * b + 8) {
            dst[b] = (uint8_t)v;
        } else {
            uint32_t mask = 0;
            for (int j = lo; j < hi; j++) mask |= 1u << (7 - (j - 8 * b));
            const uintptr_t a = (uintptr_t)(dst + b);
            uint32_t *word = (uint32_t *)(a & ~(uintptr_t)3);
            const uint32_t sh = (uint32_t)(a & 3u) * 8u;
            atomicAnd(word, ~(mask << sh));
            atomicOr(word, (v & mask) << sh);
        }
    }
}

// Word q of R and S from the packed state (25 bytes, r_0..r_99 s_0..s_99, MSB first).
__device__ __forceinline__ void quad_gather(const uint8_t *src, uint32_t q, uint32_t &r, uint32_t &s)
{
    r = 0u;
    s = 0u;
    for (uint32_t b = 0; b < 32u; b++) {
        const uint32_t i = 32u * q + b;
        if (i >= 100u) break;
        const uint32_t js = 100u + i;
        r |= ((uint32_t)(src[i >> 3] >> (7u - (i & 7u))) & 1u) << b;
        s |= ((uint32_t)(src[js >> 3] >> (7u - (js & 7u))) & 1u) << b;
    }
}

// Lane 0 of the quad packs the quad's words into 25 bytes at dst (all four lanes call it).
__device__ __forceinline__ void quad_write_back(uint32_t r, uint32_t s, uint32_t q, uint8_t *dst)
{
    const uint32_t rw[4] = {qperm<qp(0, 0, 0, 0)>(r), qperm<qp(1, 1, 1, 1)>(r), qperm<qp(2, 2, 2, 2)>(r),
                            qperm<qp(3, 3, 3, 3)>(r)};
    const uint32_t sw[4] = {qperm<qp(0, 0, 0, 0)>(s), qperm<qp(1, 1, 1, 1)>(s), qperm<qp(2, 2, 2, 2)>(s),
                            qperm<qp(3, 3, 3, 3)>(s)};
    if (q) return;
#pragma unroll
    for (int byte = 0; byte < 25; byte++) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int j = 8 * byte + k;
            const uint32_t bit = j < 100 ? (rw[j >> 5] >> (j & 31)) & 1u : (sw[(j - 100) >> 5] >> ((j - 100) & 31)) & 1u;
            v |= bit << (7 - k);
        }
        dst[byte] = (uint8_t)v;
    }
}

}  // namespace mickey
