// Device building blocks shared by the plain, batched and served kernels: input
// staging, the initialisation clocks, state load/store, and the 32-clock row-major
// delivery block.
//
// Plane layouts: a "plane" is one 32-bit word per slice (32 instances) for one clock or
// one register bit, stored contiguously over slices with a pitch of 4*nslices bytes.
#pragma once
#include "mickey_bitslice.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mickey {

constexpr int kInitClocks = 260;   // 80 IV slots + 80 key bits + 100 preclocks
constexpr int kInputPlanes = 160;  // clocks that take an input bit
constexpr int kMaskPlanes = 96;    // "lane has started" planes, clocks 0..95
constexpr uint32_t kNoRequest = 0xFFFFFFFFu;

using bitops::swap_stage;
using bitops::transpose32;
using bitops::transpose_half;

// ---------------------------------------------------------------------------------
// a1: input staging (the bitsliced input handler of Sec. IV-D).  Slot i (instance i, or
// request order[i] when ORDER) with IV length L idles for d = 80 - L clocks and then
// takes its L IV bits (MSB first), so the key always enters at clock 80 in every lane:
// its input string is the 160-bit number (ivL << 80) | key read MSB first (ivL = the
// L-bit IV), and its "started" string is d zeros then ones.  A block of 256 slots
// (8 slices) writes these strings as 32-bit chunks to LDS; then one wave turns each
// (slice, chunk) into 32 bit-planes with an in-register 32x32 transpose.
//   nslots: real slots (others are padding with an all-zero key and 80-bit IV)
//   nslices: plane pitch in words (slots are 32*nslices)
template <bool MASKED, bool ORDER>
__global__ __launch_bounds__(256) void stage_kernel(const uint8_t *__restrict__ keys,
                                                    const uint8_t *__restrict__ ivs,
                                                    const uint8_t *__restrict__ iv_bits,
                                                    const uint32_t *__restrict__ order, uint32_t nslots,
                                                    uint32_t nslices, uint32_t *__restrict__ in_planes,
                                                    uint32_t *__restrict__ mask_planes,
                                                    uint32_t *__restrict__ status)
{
    constexpr int kChunks = kInputPlanes / 32, kMaskChunks = kMaskPlanes / 32;
    __shared__ uint32_t chunk[kChunks + kMaskChunks][256];
    const uint32_t tid = threadIdx.x;
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t req = i < nslots ? i : kNoRequest;
    if (ORDER && req != kNoRequest) req = order[i];
    uint64_t kh = 0, ih = 0;
    uint32_t kl = 0, il = 0, L = 80;
    if (req != kNoRequest) {
        const uint8_t *k = keys + 10ull * req;
        const uint8_t *v = ivs + 10ull * req;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            kh = (kh << 8) | k[b];
            ih = (ih << 8) | v[b];
        }
        kl = ((uint32_t)k[8] << 8) | k[9];
        il = ((uint32_t)v[8] << 8) | v[9];
        if (MASKED) {
            L = iv_bits[req];
            if (L > 80u) {
                atomicOr(status, 1u);
                L = 80u;
            }
        }
    }
    typedef unsigned __int128 u128;
    const u128 key80 = ((u128)kh << 16) | kl;
    const u128 iv80 = ((u128)ih << 16) | il;
    const u128 ivL = L ? (iv80 >> (80u - L)) : (u128)0;
    const u128 lo = key80 | (ivL << 80);    // bits 0..127 of the input string
    chunk[0][tid] = (uint32_t)(ivL >> 48);  // bits 159..128: clocks 0..31, MSB first
    chunk[1][tid] = (uint32_t)(lo >> 96);
    chunk[2][tid] = (uint32_t)(lo >> 64);
    chunk[3][tid] = (uint32_t)(lo >> 32);
    chunk[4][tid] = (uint32_t)lo;
    if (MASKED) {
        const uint32_t d = 80u - L;  // clocks before this lane starts
#pragma unroll
        for (int c = 0; c < kMaskChunks; c++) {
            const uint32_t first = 32u * c;  // started bit of clock first+b is (first+b >= d)
            chunk[kChunks + c][tid] =
                d <= first ? 0xFFFFFFFFu : (d >= first + 32u ? 0u : (0xFFFFFFFFu >> (d - first)));
        }
    }
    __syncthreads();
    constexpr int kTasks = 8 * (kChunks + (MASKED ? kMaskChunks : 0));
    static_assert(kTasks <= 64, "one wave does the transposes");
    if (tid >= (uint32_t)kTasks) return;
    const uint32_t sl = tid & 7u, c = tid >> 3;
    const uint32_t slice = blockIdx.x * 8u + sl;
    if (slice >= nslices) return;
    uint32_t a[32];
#pragma unroll
    for (int l = 0; l < 32; l++) a[l] = chunk[c][32u * sl + l];
    transpose32(a);  // a[r] bit l = bit r of slot l's chunk word = clock 32c + 31 - r
    uint32_t *dst = c < (uint32_t)kChunks ? in_planes + (size_t)(32u * c) * nslices
                                          : mask_planes + (size_t)(32u * (c - kChunks)) * nslices;
#pragma unroll
    for (int r = 0; r < 32; r++) dst[(size_t)(31 - r) * nslices + slice] = a[r];
}

__device__ __forceinline__ uint32_t ld_plane(const uint32_t *base, size_t pitch, uint32_t t, uint32_t voff)
{
    return *(const uint32_t *)((const char *)base + (size_t)t * pitch + voff);
}

// a2: the 260 initialisation clocks of one slice from the zero state.  With MASKED,
// lanes whose IV is shorter than 80 bits stay at the zero state until their first IV
// bit (only needed when some IV length differs from 80).
template <bool MASKED, int U>
__device__ __forceinline__ void init_clocks(Regs<1> &x, const uint32_t *in_planes, const uint32_t *mask_planes,
                                            size_t pitch, uint32_t voff)
{
#pragma unroll
    for (int j = 0; j < 100; j++) {
        x.r[j].w[0] = 0u;
        x.s[j].w[0] = 0u;
    }
    const Word<1> ones = {{0xFFFFFFFFu}};
    for (uint32_t t = 0; t < 80u; t += U) {  // IV slots
        Word<1> in[U], m[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            in[u].w[0] = ld_plane(in_planes, pitch, t + u, voff);
            m[u].w[0] = MASKED ? ld_plane(mask_planes, pitch, t + u, voff) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int u = 0; u < U; u++) clock_mix<1, MASKED>(x, in[u], m[u]);
    }
    for (uint32_t t = 80u; t < 160u; t += U) {  // key bits
        Word<1> in[U];
#pragma unroll
        for (int u = 0; u < U; u++) in[u].w[0] = ld_plane(in_planes, pitch, t + u, voff);
#pragma unroll
        for (int u = 0; u < U; u++) clock_mix<1, false>(x, in[u], ones);
    }
    const Word<1> zero = {{0u}};
    for (uint32_t t = 160u; t < (uint32_t)kInitClocks; t += U) {  // 100 preclocks
#pragma unroll
        for (int u = 0; u < U; u++) clock_mix<1, false>(x, zero, ones);
    }
    static_assert(80 % U == 0 && 100 % U == 0, "unroll must divide the phase lengths");
}

template <int K>
__device__ __forceinline__ Word<K> ld_word(const char *p)
{
    Word<K> v;
    if constexpr (K == 1) {
        v.w[0] = *(const uint32_t *)p;
    } else {
        const uint2 q = *(const uint2 *)p;
        v.w[0] = q.x;
        v.w[1] = q.y;
    }
    return v;
}

template <int K>
__device__ __forceinline__ void st_word(char *p, const Word<K> &v)
{
    if constexpr (K == 1) {
        *(uint32_t *)p = v.w[0];
    } else {
        *(uint2 *)p = make_uint2(v.w[0], v.w[1]);
    }
}

// Output words always go to device memory.  Stores through pointers that were loaded
// from memory would be flat stores, which also count against the LDS wait counter, so
// every later LDS wait (the transposes) would wait for them; a global-address-space
// pointer gives global stores.
typedef __attribute__((address_space(1))) uint32_t global_u32;
__device__ __forceinline__ void store_global(uint32_t *p, uint32_t v) { *(global_u32 *)p = v; }
__device__ __forceinline__ void store_global_f32(float *p, float v)
{
    *(__attribute__((address_space(1))) float *)p = v;
}

// One keystream word (K 32-bit words) at the lane's offset in a wave-uniform plane: a
// vector buffer store whose resource is built from the scalar plane address, so that the
// per-clock address arithmetic stays on the scalar unit.
template <int K>
__device__ __forceinline__ void store_plane(char *plane, uint32_t voff, const Word<K> &v)
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(plane, (short)0, 0x7FFFFFFF, 0x00020000);
    if constexpr (K == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(v.w[0], rs, (int)voff, 0, 0);
    } else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        u32x2 d;
        d.x = v.w[0];
        d.y = v.w[1];
        __builtin_amdgcn_raw_buffer_store_b64(d, rs, (int)voff, 0, 0);
    }
}

template <int K>
__device__ __forceinline__ void load_state(Regs<K> &x, const uint32_t *state, size_t pitch, uint32_t voff)
{
#pragma unroll
    for (int j = 0; j < 100; j++) {
        x.r[j] = ld_word<K>((const char *)state + (size_t)j * pitch + voff);
        x.s[j] = ld_word<K>((const char *)state + (size_t)(100 + j) * pitch + voff);
    }
}

template <int K>
__device__ __forceinline__ void store_state(const Regs<K> &x, uint32_t *state, size_t pitch, uint32_t voff)
{
    asm volatile("" : "+v"(voff));  // keep the load addresses from living across the loop
#pragma unroll
    for (int j = 0; j < 100; j++) {
        st_word<K>((char *)state + (size_t)j * pitch + voff, x.r[j]);
        st_word<K>((char *)state + (size_t)(100 + j) * pitch + voff, x.s[j]);
    }
}

// a5: the transposition of a staged 32-clock block: row 31-b of column `col` holds the
// keystream word of clock b (bit l = instance l); emit(l, w) receives instance l's word,
// whose bit (31 - b) is clock b.  Two 16-row halves keep at most 16 words live.
template <int NT, class Emit>
__device__ __forceinline__ void rowmajor_flush(uint32_t (&zbuf)[32][NT], uint32_t col, Emit &&emit)
{
#pragma unroll
    for (int h = 0; h < 32; h += 16) {
        uint32_t a[16];
#pragma unroll
        for (int i = 0; i < 16; i++) a[i] = zbuf[h + i][col];
        transpose_half(a);
#pragma unroll
        for (int i = 0; i < 16; i++) zbuf[h + i][col] = a[i];
    }
#pragma unroll
    for (int i = 0; i < 16; i++) {
        uint32_t lo = zbuf[i][col], hi = zbuf[i + 16][col];
        swap_stage<16>(lo, hi);
        emit(i, lo);
        emit(i + 16, hi);
    }
}

// a3 + a5: 32 keystream clocks of one slice, delivered as one 32-bit word per
// instance: emit(l, w) receives w whose bit (31 - b) is keystream bit b of the block
// for instance l.  The per-clock words are staged in LDS (column `col` of zbuf, one
// 32-word column per lane) and transposed in two 16-row halves so that no more than 16
// words are live next to the 200 state registers.
template <int U, int NT, class Emit>
__device__ __forceinline__ void rowmajor_block(Regs<1> &x, uint32_t (&zbuf)[32][NT], uint32_t col, Emit &&emit)
{
    static_assert(32 % U == 0, "unroll must divide 32");
    for (int b0 = 0; b0 < 32; b0 += U) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            zbuf[31 - (b0 + u)][col] = (x.r[0] ^ x.s[0]).w[0];  // row 31-b holds clock b
            clock_gen<1>(x);
        }
    }
    rowmajor_flush(zbuf, col, emit);
}

}  // namespace mickey
