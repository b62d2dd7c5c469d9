// Bit-matrix helpers shared by the bitsliced ciphers: v_bitop3_b32 truth-table operands
// and in-register 32x32 bit transposes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bitops {

// bitop3 truth-table operands: result bit = imm[(a << 2) | (b << 1) | c].
constexpr int TA = 0xF0, TB = 0xCC, TC = 0xAA;

// Bit-matrix transposes.  The delta-swap stages below each exchange bit s of the row
// index with bit s of the column index; they commute, so a 32x32 transpose can run as
// stages 8,4,2,1 inside two 16-row halves and stage 16 last.

template <int S>
__device__ __forceinline__ void swap_stage(uint32_t &x, uint32_t &y)
{
    // rows i and i+S: x keeps its columns with bit S clear and takes y's; y the reverse
    constexpr uint32_t lo = S == 16 ? 0x0000FFFFu : S == 8 ? 0x00FF00FFu : S == 4 ? 0x0F0F0F0Fu
                          : S == 2  ? 0x33333333u : 0x55555555u;
    constexpr int sel = (TA & ~TC) | (TB & TC);  // c ? b : a
    const uint32_t nx = __builtin_amdgcn_bitop3_b32(x, y << S, ~lo, sel);
    const uint32_t ny = __builtin_amdgcn_bitop3_b32(y, x >> S, lo, sel);
    x = nx;
    y = ny;
}

// Stages 8, 4, 2, 1 on 16 consecutive rows.
__device__ __forceinline__ void transpose_half(uint32_t (&a)[16])
{
#pragma unroll
    for (int i = 0; i < 16; i++)
        if (!(i & 8)) swap_stage<8>(a[i], a[i + 8]);
#pragma unroll
    for (int i = 0; i < 16; i++)
        if (!(i & 4)) swap_stage<4>(a[i], a[i + 4]);
#pragma unroll
    for (int i = 0; i < 16; i++)
        if (!(i & 2)) swap_stage<2>(a[i], a[i + 2]);
#pragma unroll
    for (int i = 0; i < 16; i++)
        if (!(i & 1)) swap_stage<1>(a[i], a[i + 1]);
}

// Full 32x32 transpose in registers: on return a[r] bit c equals the input a[c] bit r.
__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
#pragma unroll
    for (int i = 0; i < 16; i++) swap_stage<16>(a[i], a[i + 16]);
#pragma unroll
    for (int h = 0; h < 32; h += 16) {
        uint32_t b[16];
#pragma unroll
        for (int i = 0; i < 16; i++) b[i] = a[h + i];
        transpose_half(b);
#pragma unroll
        for (int i = 0; i < 16; i++) a[h + i] = b[i];
    }
}

}  // namespace bitops
