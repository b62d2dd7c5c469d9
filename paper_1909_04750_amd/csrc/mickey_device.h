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
// L-bit IV), and its "started" string is d zeros then ones.  A block of 256 threads
// takes kStageSlices slices (32 slots each): it writes these strings as 32-bit chunks to
// LDS, then turns each (chunk, slice) into 32 bit-planes with an in-register 32x32
// transpose; a wave takes one chunk of 64 consecutive slices, so every plane store
// writes 256 contiguous bytes.
//   nslots: real slots (others are padding with an all-zero key and 80-bit IV)
//   nslices: plane pitch in words (slots are 32*nslices); the grid is
//            ceil(nslices / kStageSlices) blocks
constexpr int kStageSlices = 64;
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
    constexpr int kRows = kChunks + (MASKED ? kMaskChunks : 0);
    constexpr uint32_t kStride = 33;  // words per slice in a chunk row: the pad puts a wave's 64
                                      // column reads (one per slice) in different banks
    __shared__ uint32_t chunk[kRows][kStageSlices * kStride];
    const uint32_t tid = threadIdx.x;
    for (uint32_t j = tid; j < 32u * kStageSlices; j += 256u) {
        const uint32_t i = blockIdx.x * (32u * kStageSlices) + j;
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
        const u128 lo = key80 | (ivL << 80);  // bits 0..127 of the input string
        const uint32_t at = (j >> 5) * kStride + (j & 31u);
        chunk[0][at] = (uint32_t)(ivL >> 48);  // bits 159..128: clocks 0..31, MSB first
        chunk[1][at] = (uint32_t)(lo >> 96);
        chunk[2][at] = (uint32_t)(lo >> 64);
        chunk[3][at] = (uint32_t)(lo >> 32);
        chunk[4][at] = (uint32_t)lo;
        if constexpr (MASKED) {
            const uint32_t d = 80u - L;  // clocks before this lane starts
#pragma unroll
            for (int c = 0; c < kMaskChunks; c++) {
                const uint32_t first = 32u * c;  // started bit of clock first+b is (first+b >= d)
                chunk[kChunks + c][at] =
                    d <= first ? 0xFFFFFFFFu : (d >= first + 32u ? 0u : (0xFFFFFFFFu >> (d - first)));
            }
        }
    }
    __syncthreads();
    for (uint32_t task = tid; task < (uint32_t)(kRows * kStageSlices); task += 256u) {
        const uint32_t sl = task % kStageSlices, c = task / kStageSlices;
        const uint32_t slice = blockIdx.x * kStageSlices + sl;
        if (slice >= nslices) continue;
        uint32_t a[32];
#pragma unroll
        for (int l = 0; l < 32; l++) a[l] = chunk[c][sl * kStride + l];
        transpose32(a);  // a[r] bit l = bit r of slot l's chunk word = clock 32c + 31 - r
        uint32_t *dst = c < (uint32_t)kChunks ? in_planes + (size_t)(32u * c) * nslices
                                              : mask_planes + (size_t)(32u * (c - kChunks)) * nslices;
#pragma unroll
        for (int r = 0; r < 32; r++) dst[(size_t)(31 - r) * nslices + slice] = a[r];
    }
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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Four consecutive words; p 16-byte aligned.
__device__ __forceinline__ void store_global_x4(uint32_t *p, u32x4 v)
{
    *(__attribute__((address_space(1))) u32x4 *)p = v;
}
__device__ __forceinline__ void store_global_f32x4(float *p, f32x4 v)
{
    *(__attribute__((address_space(1))) f32x4 *)p = v;
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

// ---------------------------------------------------------------------------------
// Split clock on two waves of one workgroup (wave 0 keeps the R words, wave 1 the S
// words of the same slices).  Each clock the waves swap r_33, s_34 and s_0 through a
// double-buffered LDS slot with one LDS-only barrier: a wave writes its value as soon as
// its half-clock has made it final and reads the other's right after the barrier, so the
// round trip overlaps the rest of the half-clock.  The slot a clock writes is read again
// only two clocks later, after another barrier.  Both waves must run the same number of
// clocks (one barrier each).
struct SplitLds {
    uint32_t r33[2][64];
    uint32_t s34[2][64];
    uint32_t s0[2][64];
};

// Barrier for LDS traffic only (output stores stay in flight).  The caller issues its
// LDS reads right after it and then fences the scheduler, so that the reads go out
// before the half-clock's ALU work rather than wherever the scheduler would put them.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One clock of the R wave; s34/s0 hold the current state's s_34 and s_0 and are replaced
// by the next state's.  `ph` is the exchange buffer of the next state.
__device__ __forceinline__ void split_r_clock(Regs<1> &x, Word<1> &s34, Word<1> &s0, SplitLds &xl,
                                              uint32_t lane, int ph)
{
    const Word<1> cr = s34 ^ x.r[67];
    const Word<1> fbr = x.r[99];
    r_upper<1>(x, cr, fbr);
    xl.r33[ph][lane] = x.r[kRCut].w[0];
    lds_barrier();
    s34.w[0] = xl.s34[ph][lane];
    s0.w[0] = xl.s0[ph][lane];
    __builtin_amdgcn_sched_barrier(0);
    r_lower<1>(x, cr, fbr);
    // The LDS round trip is hidden behind r_lower: keep the next clock's work from moving
    // in front of the wait for it.
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" : "+v"(s34.w[0]), "+v"(s0.w[0]));
}

__device__ __forceinline__ void split_s_clock(Regs<1> &x, Word<1> &r33, SplitLds &xl, uint32_t lane, int ph)
{
    const Word<1> cs = x.s[67] ^ r33;
    const Word<1> fbs = x.s[99];
    const Word<1> g1 = fbs & cs;
    const Word<1> g0 = fbs ^ g1;
    Word<1> prev = x.s[0];
    s_lower<1>(x, prev, fbs, g0, g1);
    xl.s34[ph][lane] = x.s[kSCut].w[0];
    xl.s0[ph][lane] = fbs.w[0];  // the next s_0
    lds_barrier();
    r33.w[0] = xl.r33[ph][lane];
    __builtin_amdgcn_sched_barrier(0);
    s_upper<1>(x, prev, fbs, g0, g1);
    __builtin_amdgcn_sched_barrier(0);  // c_S of the next clock waits for r_33 only here
}

// The S wave's clock as a descending sweep (s_99..s_34 before the exchange, s_33..s_1
// after); alternated with split_s_clock it keeps the S words in one register set.
__device__ __forceinline__ void split_s_clock_desc(Regs<1> &x, Word<1> &r33, SplitLds &xl, uint32_t lane, int ph)
{
    const Word<1> cs = x.s[67] ^ r33;
    const Word<1> fbs = x.s[99];
    const Word<1> g1 = fbs & cs;
    const Word<1> g0 = fbs ^ g1;
    Word<1> nxt;
    s_upper_desc<1>(x, nxt, fbs, g0, g1);
    xl.s34[ph][lane] = x.s[kSCut].w[0];
    xl.s0[ph][lane] = fbs.w[0];  // the next s_0
    lds_barrier();
    r33.w[0] = xl.r33[ph][lane];
    __builtin_amdgcn_sched_barrier(0);
    s_lower_desc<1>(x, nxt, fbs, g0, g1);
    __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------------------------------
// Four-wave split clock (one workgroup of four waves per 64 slices): wave 0 keeps
// r_0..r_49, wave 1 r_50..r_99, wave 2 s_0..s_49, wave 3 s_50..s_99.  Each position's
// next value is a function of the current state (r_next / s_next), so each wave first
// computes the values the others need for the next clock, writes them to a
// double-buffered LDS slot, passes the clock's one barrier, issues its reads, and then
// computes the rest of its half-register.  Exchanged per clock (next-state values): r_49
// (to wave 1), r_33 (to the S waves, for c_S), r_99 and r_67 (to wave 0, for fb_R and
// c_R), s_34 (to the R waves), s_0 (to wave 0, for z), s_49 (to wave 3), s_50, s_99 and
// s_67 (to wave 2).
enum : int { kX_R49, kX_R33, kX_R99, kX_R67, kX_S49, kX_S34, kX_S0, kX_S50, kX_S99, kX_S67, kXSlots };
struct Split4Lds {
    uint32_t v[2][kXSlots][64];
};

constexpr bool ex3(int i, int a, int b, int c) { return i == a || i == b || i == c; }

// n.r[LO + j] for j < N, except positions A, B, C
template <int LO, int A, int B, int C, int... J>
__device__ __forceinline__ void r_next_range(Regs<1> &n, const Regs<1> &x, const Word<1> &cr, const Word<1> &fbr,
                                             std::integer_sequence<int, J...>)
{
    ((ex3(LO + J, A, B, C) ? void() : void(n.r[LO + J] = r_next<LO + J, 1>(x, cr, fbr))), ...);
}
template <int LO, int A, int B, int C, int... J>
__device__ __forceinline__ void s_next_range(Regs<1> &n, const Regs<1> &x, const Word<1> &fbs, const Word<1> &g0,
                                             const Word<1> &g1, std::integer_sequence<int, J...>)
{
    ((ex3(LO + J, A, B, C) ? void() : void(n.s[LO + J] = s_next<LO + J, 1>(x, fbs, g0, g1))), ...);
}

struct S4In {  // next-clock values a wave receives
    Word<1> a, b, c, d;
};

// wave 0: in = {r_99, r_67, s_34, s_0} of the current state
template <int PH>
__device__ __forceinline__ void s4_clock_rlo(Regs<1> &x, S4In &in, Split4Lds &xl, uint32_t lane)
{
    const Word<1> cr = in.c ^ in.b, fbr = in.a;
    Regs<1> n;
    n.r[49] = r_next<49, 1>(x, cr, fbr);
    n.r[33] = r_next<33, 1>(x, cr, fbr);
    xl.v[PH][kX_R49][lane] = n.r[49].w[0];
    xl.v[PH][kX_R33][lane] = n.r[33].w[0];
    lds_barrier();
    in.a.w[0] = xl.v[PH][kX_R99][lane];
    in.b.w[0] = xl.v[PH][kX_R67][lane];
    in.c.w[0] = xl.v[PH][kX_S34][lane];
    in.d.w[0] = xl.v[PH][kX_S0][lane];
    __builtin_amdgcn_sched_barrier(0);
    r_next_range<0, 49, 33, -1>(n, x, cr, fbr, std::make_integer_sequence<int, 50>{});
#pragma unroll
    for (int j = 0; j < 50; j++) x.r[j] = n.r[j];
    __builtin_amdgcn_sched_barrier(0);
}

// wave 1: in = {s_34}; x.r[49] holds the current r_49
template <int PH>
__device__ __forceinline__ void s4_clock_rhi(Regs<1> &x, S4In &in, Split4Lds &xl, uint32_t lane)
{
    const Word<1> cr = in.a ^ x.r[67], fbr = x.r[99];
    Regs<1> n;
    n.r[99] = r_next<99, 1>(x, cr, fbr);
    n.r[67] = r_next<67, 1>(x, cr, fbr);
    xl.v[PH][kX_R99][lane] = n.r[99].w[0];
    xl.v[PH][kX_R67][lane] = n.r[67].w[0];
    lds_barrier();
    Word<1> r49;
    r49.w[0] = xl.v[PH][kX_R49][lane];
    in.a.w[0] = xl.v[PH][kX_S34][lane];
    __builtin_amdgcn_sched_barrier(0);
    r_next_range<50, 99, 67, -1>(n, x, cr, fbr, std::make_integer_sequence<int, 50>{});
#pragma unroll
    for (int j = 50; j < 100; j++) x.r[j] = n.r[j];
    x.r[49] = r49;
    __builtin_amdgcn_sched_barrier(0);
}

// wave 2: in = {s_99, s_67, r_33}; x.s[50] holds the current s_50
template <int PH>
__device__ __forceinline__ void s4_clock_slo(Regs<1> &x, S4In &in, Split4Lds &xl, uint32_t lane)
{
    const Word<1> cs = in.b ^ in.c, fbs = in.a;
    const Word<1> g1 = fbs & cs;
    const Word<1> g0 = fbs ^ g1;
    Regs<1> n;
    n.s[49] = s_next<49, 1>(x, fbs, g0, g1);
    n.s[34] = s_next<34, 1>(x, fbs, g0, g1);
    xl.v[PH][kX_S49][lane] = n.s[49].w[0];
    xl.v[PH][kX_S34][lane] = n.s[34].w[0];
    xl.v[PH][kX_S0][lane] = fbs.w[0];  // the next s_0
    lds_barrier();
    Word<1> s50;
    s50.w[0] = xl.v[PH][kX_S50][lane];
    in.a.w[0] = xl.v[PH][kX_S99][lane];
    in.b.w[0] = xl.v[PH][kX_S67][lane];
    in.c.w[0] = xl.v[PH][kX_R33][lane];
    __builtin_amdgcn_sched_barrier(0);
    s_next_range<0, 49, 34, -1>(n, x, fbs, g0, g1, std::make_integer_sequence<int, 50>{});
#pragma unroll
    for (int j = 0; j < 50; j++) x.s[j] = n.s[j];
    x.s[50] = s50;
    __builtin_amdgcn_sched_barrier(0);
}

// wave 3: in = {r_33}; x.s[49] holds the current s_49
template <int PH>
__device__ __forceinline__ void s4_clock_shi(Regs<1> &x, S4In &in, Split4Lds &xl, uint32_t lane)
{
    const Word<1> cs = x.s[67] ^ in.a, fbs = x.s[99];
    const Word<1> g1 = fbs & cs;
    const Word<1> g0 = fbs ^ g1;
    Regs<1> n;
    n.s[50] = s_next<50, 1>(x, fbs, g0, g1);
    n.s[99] = s_next<99, 1>(x, fbs, g0, g1);
    n.s[67] = s_next<67, 1>(x, fbs, g0, g1);
    xl.v[PH][kX_S50][lane] = n.s[50].w[0];
    xl.v[PH][kX_S99][lane] = n.s[99].w[0];
    xl.v[PH][kX_S67][lane] = n.s[67].w[0];
    lds_barrier();
    Word<1> s49;
    s49.w[0] = xl.v[PH][kX_S49][lane];
    in.a.w[0] = xl.v[PH][kX_R33][lane];
    __builtin_amdgcn_sched_barrier(0);
    s_next_range<50, 50, 99, 67>(n, x, fbs, g0, g1, std::make_integer_sequence<int, 50>{});
#pragma unroll
    for (int j = 50; j < 100; j++) x.s[j] = n.s[j];
    x.s[49] = s49;
    __builtin_amdgcn_sched_barrier(0);
}

// ---------------------------------------------------------------------------------
// a5, staged: tiled transpose of bit-planes (plane t: one word per slice, nslices words)
// into per-instance row words.  A 256-thread workgroup takes a tile of kTpSlices slices
// (512 instances) x kTpClocks clocks: it reads the tile's plane words into LDS, turns
// every (slice, 32-clock block) pair into 32 row words with an in-register 32x32
// transpose, and leaves row i (instance 32*s0 + i) of the tile in LDS, its block-q word
// at tile_row_word(lds, i, q): bit 31 - b is clock t0 + 32q + b.
constexpr int kTpSlices = 16;                     // slices per tile
constexpr int kTpBlocks = 32;                     // 32-clock blocks per tile
constexpr int kTpClocks = 32 * kTpBlocks;
constexpr int kTpInStride = 32 * kTpSlices + 16;  // LDS words per block; the pad puts
                                                  // adjacent blocks in other banks
constexpr int kTpLdsWords = kTpBlocks * kTpInStride;
static_assert(32 * kTpSlices * kTpBlocks <= kTpLdsWords, "row staging reuses the tile");

// nb (<= kTpBlocks) blocks from clock t0, slices s0 .. s0+15 (those past nslices read a
// copy of the last pair and must not be written out; nslices is even).  Ends with the
// rows in LDS after a barrier.
// `publish` runs after the plane reads are issued and before the first barrier: a caller's
// own LDS writes there are visible to the whole block afterwards.
template <class Publish>
__device__ __forceinline__ void tile_to_rows(uint32_t *lds, const uint32_t *__restrict__ planes, uint32_t nslices,
                                             uint32_t s0, uint32_t t0, uint32_t nb, uint32_t tid, Publish &&publish)
{
    {  // each lane loads a pair of slice words of one plane; 32 planes (one block) per pass
        const uint32_t pr = tid & 7u, b = tid >> 3;
        uint32_t sp = s0 + 2u * pr;
        if (sp >= nslices) sp = nslices - 2u;
        const uint32_t *src = planes + (size_t)(t0 + b) * nslices + sp;
        uint32_t *dst = lds + b * kTpSlices + 2u * pr;
        uint32_t q = 0;
        for (; q + 16u <= nb; q += 16u) {  // sixteen loads in flight before the first LDS write
            uint2 v[16];
#pragma unroll
            for (int k = 0; k < 16; k++) v[k] = *(const uint2 *)(src + (size_t)(q + k) * 32u * nslices);
#pragma unroll
            for (int k = 0; k < 16; k++) {
                dst[(q + k) * kTpInStride] = v[k].x;
                dst[(q + k) * kTpInStride + 1] = v[k].y;
            }
        }
        for (; q < nb; q++) {
            const uint2 v = *(const uint2 *)(src + (size_t)q * 32u * nslices);
            dst[q * kTpInStride] = v.x;
            dst[q * kTpInStride + 1] = v.y;
        }
    }
    publish();
    __syncthreads();
    // item (slice s, block q): row 31-b holds clock 32q+b, so the transposed word l is
    // instance l's word with bit 31-b = clock b
    uint32_t a[2][32];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t item = tid + 256u * h, s = item & 15u, q = item >> 4;
        if (q < nb) {
#pragma unroll
            for (int b = 0; b < 32; b++) a[h][31 - b] = lds[q * kTpInStride + b * kTpSlices + s];
            transpose32(a[h]);
        }
    }
    __syncthreads();
    // row 32s+l, block q at column q ^ s (the swizzle spreads a row's readers over banks)
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t item = tid + 256u * h, s = item & 15u, q = item >> 4;
        if (q < nb) {
#pragma unroll
            for (int l = 0; l < 32; l++) lds[(32u * s + l) * 32u + (q ^ s)] = a[h][l];
        }
    }
    __syncthreads();
}

// Workgroups are dealt to the 8 XCDs round-robin by linear id, and each XCD has its own
// L2.  xcd_grouped(lin, n) is a permutation of 0..n-1 that gives each XCD a contiguous run
// of logical indices, so neighbouring transpose tiles, which read the two halves of the
// same 128 B lines (16 slices are 64 B of a plane), run on one XCD and fetch each line once.
__device__ __forceinline__ uint32_t xcd_grouped(uint32_t lin, uint32_t n)
{
    constexpr uint32_t kXcds = 8;
    const uint32_t q = n / kXcds, r = n % kXcds, x = lin % kXcds;
    return x * q + (x < r ? x : r) + lin / kXcds;
}

// (tile, clock block) of this workgroup of a transpose grid, XCD-grouped.
__device__ __forceinline__ uint2 tile_of_block()
{
    const uint32_t gx = gridDim.x;
    const uint32_t l = xcd_grouped(blockIdx.x + blockIdx.y * gx, gx * gridDim.y);
    return make_uint2(l % gx, l / gx);
}

__device__ __forceinline__ uint32_t tile_row_word(const uint32_t *lds, uint32_t i, uint32_t q)
{
    return lds[i * 32u + (q ^ (i >> 5))];
}

}  // namespace mickey
