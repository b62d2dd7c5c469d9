// HIP kernels and C-ABI of the MICKEY-128 2.0 generator in libmickey.so (gfx950).
//
// Data layout in HBM (n_pad = 2048*ceil(n/2048) instances, nslices = n_pad/32, a
// multiple of 64 so that every workgroup serves 64 whole slices):
//   state   320 planes x nslices u32: plane j < 160 is r_j, plane 160+j is s_j; bit l of
//           word g is instance 32g+l.  Planes are contiguous (pitch nslices*4 bytes).
//   input   256 planes of input bits (IV part right-aligned to clock 128, then the key)
//           and 128 planes of "lane has started" masks, same shape; temporary.
//   output  bit-planes: plane t holds z_t of every instance, n_pad bits, LSB first.
// Execution: a workgroup of two waves serves 64 slices.  Wave 0 keeps the 64 slices' R
// words, wave 1 their S words, each in VGPRs for the whole call.  Per clock the waves
// meet at one barrier and swap, through a double-buffered LDS slot, the next-state values
// the other needs: R sends r_53 (for c_S); S sends s_54 (for c_R), s_0 (for z, which the R
// wave forms and stores) and, while initialising, s_80 (mixing).  Each wave writes its
// values as soon as its own sweep has made them final (R after r_159..r_53, S after
// s_1..s_54, or s_1..s_80 while initialising), and reads the other's right after the
// barrier, so the LDS round trip overlaps the rest of its half-clock.
#include "mickey128_bitslice.h"
#include "mickey_device.h"
#include "mickey_host.h"

#include "../../include/mickey128.h"

#include <hip/hip_runtime.h>

#include <new>

using namespace mickey128;
using namespace mickey_host;

namespace {

constexpr int kIvMax = 128, kKeyBits = 128;
constexpr int kInputPlanes = kIvMax + kKeyBits;  // clocks that take an input bit
constexpr int kMaskPlanes = kIvMax;              // clocks before which a lane may idle
constexpr int kInitClocks = kInputPlanes + kN;   // + 160 preclocks
constexpr uint64_t kSlicesPerGroup = 64;

struct XLds {
    uint32_t r53[2][64];
    uint32_t s54[2][64];
    uint32_t s0[2][64];
    uint32_t s80[2][64];
};

// ------------------------------------------------------------------------ staging
// a1 for 128-bit keys: instance i with IV length L idles for d = 128 - L clocks, then
// takes its L IV bits (MSB first) and the 128 key bits, so its input string is the
// 256-bit number (ivL << 128) | key read MSB first.  A workgroup of 256 threads (8
// slices) writes these strings to LDS as 32-bit chunks (bit 31-j = clock 32c+j), then
// 96 threads turn each (slice, chunk) into 32 planes with a 32x32 transpose.
__global__ __launch_bounds__(256) void m128_stage_kernel(const uint8_t *__restrict__ keys,
                                                         const uint8_t *__restrict__ ivs,
                                                         const uint8_t *__restrict__ iv_bits, uint32_t n,
                                                         uint32_t nslices, uint32_t *__restrict__ in_planes,
                                                         uint32_t *__restrict__ mask_planes,
                                                         uint32_t *__restrict__ status)
{
    constexpr int kChunks = kInputPlanes / 32, kMaskChunks = kMaskPlanes / 32;
    __shared__ uint32_t chunk[kChunks + kMaskChunks][256];
    const uint32_t tid = threadIdx.x;
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t kw[4] = {0, 0, 0, 0}, vw[4] = {0, 0, 0, 0};
    uint32_t L = kIvMax;
    if (i < n) {
        const uint8_t *k = keys + 16ull * i;
        const uint8_t *v = ivs + 16ull * i;
#pragma unroll
        for (int w = 0; w < 4; w++) {
#pragma unroll
            for (int b = 0; b < 4; b++) {
                kw[w] = (kw[w] << 8) | k[4 * w + b];
                vw[w] = (vw[w] << 8) | v[4 * w + b];
            }
        }
        if (iv_bits) {
            L = iv_bits[i];
            if (L > (uint32_t)kIvMax) {
                atomicOr(status, 1u);
                L = kIvMax;
            }
        }
    }
    // IV part: the 128-bit IV shifted right by d = 128 - L (its first L bits end at clock
    // 127), as four words, most significant first
    const uint32_t d = kIvMax - L;
    uint32_t iw[4];
#pragma unroll
    for (int w = 0; w < 4; w++) {
        // word w of (iv >> d): bits 32w .. 32w+31 from the top
        const int hi = 32 * w - (int)d;  // index (from the top) of this word's first bit in the IV
        uint32_t val = 0;
#pragma unroll
        for (int s = 0; s < 4; s++) {
            // contribution of IV word s (its bits start at 32s from the top)
            const int off = 32 * s - hi;  // shift right by off (>0) or left by -off
            if (off >= 32 || off <= -32) continue;
            val |= off >= 0 ? (vw[s] >> off) : (vw[s] << -off);
        }
        iw[w] = d >= 128u ? 0u : val;
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
        chunk[w][tid] = iw[w];
        chunk[4 + w][tid] = kw[w];
    }
#pragma unroll
    for (int c = 0; c < kMaskChunks; c++) {
        const uint32_t first = 32u * c;  // lane started at clock first+j iff first+j >= d
        chunk[kChunks + c][tid] = d <= first ? 0xFFFFFFFFu : (d >= first + 32u ? 0u : (0xFFFFFFFFu >> (d - first)));
    }
    __syncthreads();
    constexpr int kTasks = 8 * (kChunks + kMaskChunks);
    if (tid >= (uint32_t)kTasks) return;
    const uint32_t sl = tid & 7u, c = tid >> 3;
    const uint32_t slice = blockIdx.x * 8u + sl;
    if (slice >= nslices) return;
    uint32_t a[32];
#pragma unroll
    for (int l = 0; l < 32; l++) a[l] = chunk[c][sl * 32u + l];
    bitops::transpose32(a);  // a[r] bit l = instance l's chunk bit r, i.e. clock 32c + 31 - r
    uint32_t *dst = c < (uint32_t)kChunks ? in_planes + (size_t)(32u * c) * nslices
                                          : mask_planes + (size_t)(32u * (c - kChunks)) * nslices;
#pragma unroll
    for (int j = 0; j < 32; j++) dst[(size_t)j * nslices + slice] = a[31 - j];
}

// ------------------------------------------------------------------------ init
// a2: registers cleared, then 416 mixing clocks: 128 clocks that take the (right-aligned)
// IV bits under the start masks, 128 key clocks, 160 preclocks with input 0.

// One R-wave init clock; s54/s80 hold the current state's values and are replaced by the
// next state's from buffer PH.
template <int PH>
__device__ __forceinline__ void r_init_clock(RRegs &x, uint32_t in, uint32_t &s54, uint32_t &s80, XLds &xl,
                                             uint32_t lane)
{
    const uint32_t cr = s54 ^ x.r[kCtlRR];
    const uint32_t fbr = b3<TA ^ TB ^ TC>(x.r[kN - 1], in, s80);
    r_range<kN - 1, kCtlSR>(x, cr, fbr);
    xl.r53[PH][lane] = x.r[kCtlSR];
    mickey::lds_barrier();
    s54 = xl.s54[PH][lane];
    s80 = xl.s80[PH][lane];
    __builtin_amdgcn_sched_barrier(0);
    r_range<kCtlSR - 1, 0>(x, cr, fbr);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" : "+v"(s54), "+v"(s80));
}

template <int PH, bool MASKED>
__device__ __forceinline__ void s_init_clock(SRegs &x, uint32_t in, uint32_t m, uint32_t &r53, XLds &xl,
                                             uint32_t lane)
{
    const uint32_t cs = x.s[kCtlSS] ^ r53;
    const uint32_t fbs = x.s[kN - 1] ^ in;
    const uint32_t g1 = fbs & cs;
    const uint32_t g0 = fbs ^ g1;
    if constexpr (PH == 1) {  // ascending: s_1..s_80 before the exchange
        uint32_t prev = x.s[0];
        s_range<1, kMixS, MASKED>(x, prev, fbs, g0, g1, m);
        xl.s54[PH][lane] = x.s[kCtlRS];
        xl.s80[PH][lane] = x.s[kMixS];
        mickey::lds_barrier();
        r53 = xl.r53[PH][lane];
        __builtin_amdgcn_sched_barrier(0);
        s_range<kMixS + 1, kN - 2, MASKED>(x, prev, fbs, g0, g1, m);
        s_top(x, prev, fbs, g0, g1);
    } else {  // descending: s_159..s_54 before the exchange
        uint32_t nxt = s_top_desc(x, fbs, g0, g1);
        s_range_desc<kN - 2, kCtlRS, MASKED>(x, nxt, fbs, g0, g1, m);
        xl.s54[PH][lane] = x.s[kCtlRS];
        xl.s80[PH][lane] = x.s[kMixS];
        mickey::lds_barrier();
        r53 = xl.r53[PH][lane];
        __builtin_amdgcn_sched_barrier(0);
        s_range_desc<kCtlRS - 1, 1, MASKED>(x, nxt, fbs, g0, g1, m);
        x.s[0] = fbs;
    }
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ uint32_t plane_word(const uint32_t *planes, uint32_t t, uint32_t nslices, uint32_t g)
{
    return planes[(size_t)t * nslices + g];
}

// Clocks t0..t1-1 (t0 even, t1 - t0 even) of the R wave; inputs come from `in_planes`
// (or are 0 when INPUT is false), loaded two clocks ahead.
template <bool INPUT>
__device__ __forceinline__ void r_init_run(RRegs &x, const uint32_t *in_planes, uint32_t nslices, uint32_t g,
                                           uint32_t t0, uint32_t t1, uint32_t &s54, uint32_t &s80, XLds &xl,
                                           uint32_t lane)
{
    uint32_t a = INPUT ? plane_word(in_planes, t0, nslices, g) : 0u;
    uint32_t b = INPUT ? plane_word(in_planes, t0 + 1, nslices, g) : 0u;
    for (uint32_t t = t0; t < t1; t += 2) {
        uint32_t na = 0, nb = 0;
        if (INPUT && t + 2 < t1) {
            na = plane_word(in_planes, t + 2, nslices, g);
            nb = plane_word(in_planes, t + 3, nslices, g);
        }
        r_init_clock<1>(x, a, s54, s80, xl, lane);
        r_init_clock<0>(x, b, s54, s80, xl, lane);
        a = na;
        b = nb;
    }
}

template <bool INPUT, bool MASKED>
__device__ __forceinline__ void s_init_run(SRegs &x, const uint32_t *in_planes, const uint32_t *mask_planes,
                                           uint32_t nslices, uint32_t g, uint32_t t0, uint32_t t1, uint32_t &r53,
                                           XLds &xl, uint32_t lane)
{
    uint32_t a = INPUT ? plane_word(in_planes, t0, nslices, g) : 0u;
    uint32_t b = INPUT ? plane_word(in_planes, t0 + 1, nslices, g) : 0u;
    uint32_t ma = MASKED ? plane_word(mask_planes, t0, nslices, g) : ~0u;
    uint32_t mb = MASKED ? plane_word(mask_planes, t0 + 1, nslices, g) : ~0u;
    for (uint32_t t = t0; t < t1; t += 2) {
        uint32_t na = 0, nb = 0, nma = ~0u, nmb = ~0u;
        if (INPUT && t + 2 < t1) {
            na = plane_word(in_planes, t + 2, nslices, g);
            nb = plane_word(in_planes, t + 3, nslices, g);
            if (MASKED) {
                nma = plane_word(mask_planes, t + 2, nslices, g);
                nmb = plane_word(mask_planes, t + 3, nslices, g);
            }
        }
        s_init_clock<1, MASKED>(x, a, ma, r53, xl, lane);
        s_init_clock<0, MASKED>(x, b, mb, r53, xl, lane);
        a = na;
        b = nb;
        ma = nma;
        mb = nmb;
    }
}

// The buffer a clock writes (PH = 1 on even clocks) is read again only two clocks later,
// after every wave has passed the barrier in between, so one barrier per clock suffices.
__global__ __launch_bounds__(128) void m128_init_kernel(const uint32_t *__restrict__ in_planes,
                                                        const uint32_t *__restrict__ mask_planes,
                                                        uint32_t *__restrict__ state, uint32_t nslices)
{
    __shared__ XLds xl;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * 64u + lane;  // nslices is a multiple of 64
    const size_t pitch = (size_t)nslices;
    if (wave == 0) {
        RRegs x;
#pragma unroll
        for (int j = 0; j < kN; j++) x.r[j] = 0u;
        xl.r53[0][lane] = 0u;
        mickey::lds_barrier();
        uint32_t s54 = xl.s54[0][lane], s80 = xl.s80[0][lane];
        __builtin_amdgcn_sched_barrier(0);
        r_init_run<true>(x, in_planes, nslices, g, 0, kInputPlanes, s54, s80, xl, lane);
        r_init_run<false>(x, in_planes, nslices, g, kInputPlanes, kInitClocks, s54, s80, xl, lane);
#pragma unroll
        for (int j = 0; j < kN; j++) state[(size_t)j * pitch + g] = x.r[j];
    } else {
        SRegs x;
#pragma unroll
        for (int j = 0; j < kN; j++) x.s[j] = 0u;
        xl.s54[0][lane] = 0u;
        xl.s80[0][lane] = 0u;
        mickey::lds_barrier();
        uint32_t r53 = xl.r53[0][lane];
        __builtin_amdgcn_sched_barrier(0);
        s_init_run<true, true>(x, in_planes, mask_planes, nslices, g, 0, kMaskPlanes, r53, xl, lane);
        s_init_run<true, false>(x, in_planes + (size_t)kMaskPlanes * nslices, mask_planes, nslices, g, 0,
                                kInputPlanes - kMaskPlanes, r53, xl, lane);
        s_init_run<false, false>(x, in_planes, mask_planes, nslices, g, kInputPlanes, kInitClocks, r53, xl, lane);
#pragma unroll
        for (int j = 0; j < kN; j++) state[(size_t)(kN + j) * pitch + g] = x.s[j];
    }
}

// ------------------------------------------------------------------------ generate
// a3 + a4 + a6: keystream clocks, one bit-plane word per clock from the R wave (z = r_0 ^
// s_0 of the state before the clock), state write-back at the end.

template <int PH>
__device__ __forceinline__ void r_gen_clock(RRegs &x, uint32_t &s54, uint32_t &s0, XLds &xl, uint32_t lane)
{
    const uint32_t cr = s54 ^ x.r[kCtlRR];
    const uint32_t fbr = x.r[kN - 1];
    r_range<kN - 1, kCtlSR>(x, cr, fbr);
    xl.r53[PH][lane] = x.r[kCtlSR];
    mickey::lds_barrier();
    s54 = xl.s54[PH][lane];
    s0 = xl.s0[PH][lane];
    __builtin_amdgcn_sched_barrier(0);
    r_range<kCtlSR - 1, 0>(x, cr, fbr);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("" : "+v"(s54), "+v"(s0));
}

template <int PH>
__device__ __forceinline__ void s_gen_clock(SRegs &x, uint32_t &r53, XLds &xl, uint32_t lane)
{
    const uint32_t cs = x.s[kCtlSS] ^ r53;
    const uint32_t fbs = x.s[kN - 1];
    const uint32_t g1 = fbs & cs;
    const uint32_t g0 = fbs ^ g1;
    if constexpr (PH == 1) {  // ascending: s_1..s_54 before the exchange
        uint32_t prev = x.s[0];
        s_range<1, kCtlRS, false>(x, prev, fbs, g0, g1, 0u);
        xl.s54[PH][lane] = x.s[kCtlRS];
        xl.s0[PH][lane] = fbs;  // the next s_0
        mickey::lds_barrier();
        r53 = xl.r53[PH][lane];
        __builtin_amdgcn_sched_barrier(0);
        s_range<kCtlRS + 1, kN - 2, false>(x, prev, fbs, g0, g1, 0u);
        s_top(x, prev, fbs, g0, g1);
    } else {  // descending: s_159..s_54 before the exchange
        uint32_t nxt = s_top_desc(x, fbs, g0, g1);
        s_range_desc<kN - 2, kCtlRS, false>(x, nxt, fbs, g0, g1, 0u);
        xl.s54[PH][lane] = x.s[kCtlRS];
        xl.s0[PH][lane] = fbs;
        mickey::lds_barrier();
        r53 = xl.r53[PH][lane];
        __builtin_amdgcn_sched_barrier(0);
        s_range_desc<kCtlRS - 1, 1, false>(x, nxt, fbs, g0, g1, 0u);
        x.s[0] = fbs;
    }
    __builtin_amdgcn_sched_barrier(0);
}

#define M128_LOOP_R(i) x.r[i]
#define M128_LOOP_S(i) x.s[i]
#include "mickey128_loops.inc"

__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3, 3))) void m128_gen_kernel(uint32_t *__restrict__ state, uint32_t nslices,
                                                       uint64_t nbits, uint32_t *__restrict__ out)
{
    __shared__ XLds xl;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * 64u + lane;
    const size_t pitch = (size_t)nslices;
    const uint32_t xaddr = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)&xl.r53[0][lane];
    if (wave == 0) {
        RRegs x;
#pragma unroll
        for (int j = 0; j < kN; j++) x.r[j] = state[(size_t)j * pitch + g];
        xl.r53[0][lane] = x.r[kCtlSR];
        mickey::lds_barrier();
        uint32_t s54 = xl.s54[0][lane], s0 = xl.s0[0][lane];
        __builtin_amdgcn_sched_barrier(0);
        const size_t pbytes = pitch * 4u;
        const uint32_t voff = g * 4u;
        char *plane = (char *)out;  // wave-uniform
        // clock pairs: the generated R loop of mickey128_loops.inc (the clocks of
        // r_gen_clock<1>, r_gen_clock<0> with their plane stores; the buffer resource of the
        // stores is built in s[20:23])
        uint64_t npairs = nbits / 2;
        while (npairs) {
            const uint32_t iters = npairs > (1ull << 30) ? (1u << 30) : (uint32_t)npairs;
            const uint64_t base = (uint64_t)(uintptr_t)plane;
            asm volatile("s_mov_b32 s20, %[lo]\n\ts_and_b32 s21, %[hi], 0xffff\n\ts_mov_b32 s22, 0x7fffffff\n\t"
                         "s_mov_b32 s23, 0x20000\n\ts_mov_b32 s24, %[it]\n1:\n\t" M128_R_LOOP_BODY
                         "\n\ts_sub_u32 s24, s24, 1\n\ts_cmp_lg_u32 s24, 0\n\ts_cbranch_scc1 1b"
                         : M128_R_LOOP_STATE(M128_LOOP_R, s54, s0)
                         : [lo] "s"((uint32_t)base), [hi] "s"((uint32_t)(base >> 32)), [pitch] "s"((uint32_t)pbytes),
                           [it] "s"(iters), [voff] "v"(voff), [xaddr] "v"(xaddr)
                         : M128_R_LOOP_CLOBBERS, "s20", "s21", "s22", "s23", "s24", "scc", "memory");
            npairs -= iters;
            plane += (uint64_t)iters * 2 * pbytes;
        }
        if (nbits & 1) {
            mickey::store_plane<1>(plane, voff, {{x.r[0] ^ s0}});
            r_gen_clock<1>(x, s54, s0, xl, lane);
        }
        uint32_t v = voff;
        asm volatile("" : "+v"(v));  // keep the load addresses from living across the loop
#pragma unroll
        for (int j = 0; j < kN; j++) *(uint32_t *)((char *)state + (size_t)j * pbytes + v) = x.r[j];
    } else {
        SRegs x;
#pragma unroll
        for (int j = 0; j < kN; j++) x.s[j] = state[(size_t)(kN + j) * pitch + g];
        xl.s54[0][lane] = x.s[kCtlRS];
        xl.s0[0][lane] = x.s[0];
        mickey::lds_barrier();
        uint32_t r53 = xl.r53[0][lane];
        __builtin_amdgcn_sched_barrier(0);
        // clock pairs: the generated S loop of mickey128_loops.inc (the clocks of
        // s_gen_clock<1>, s_gen_clock<0>), as many iterations as the R wave's
        uint64_t npairs = nbits / 2;
        while (npairs) {
            const uint32_t iters = npairs > (1ull << 30) ? (1u << 30) : (uint32_t)npairs;
            asm volatile("s_mov_b32 s24, %[it]\n1:\n\t" M128_S_LOOP_BODY
                         "\n\ts_sub_u32 s24, s24, 1\n\ts_cmp_lg_u32 s24, 0\n\ts_cbranch_scc1 1b"
                         : M128_S_LOOP_STATE(M128_LOOP_S, r53)
                         : [it] "s"(iters), [xaddr] "v"(xaddr)
                         : M128_S_LOOP_CLOBBERS, "s24", "scc", "memory");
            npairs -= iters;
        }
        if (nbits & 1) s_gen_clock<1>(x, r53, xl, lane);
        uint32_t v = g * 4u;
        asm volatile("" : "+v"(v));
#pragma unroll
        for (int j = 0; j < kN; j++) *(uint32_t *)((char *)state + (size_t)(kN + j) * pitch * 4u + v) = x.s[j];
    }
}

}  // namespace

// ------------------------------------------------------------------------ host side

struct mickey128_state {
    size_t n = 0, n_pad = 0, nslices = 0;
    uint32_t *planes = nullptr;       // device, 320 * nslices words
    uint32_t *stage = nullptr;        // device, input + mask planes + status word
    uint32_t *host_status = nullptr;  // pinned
    hipStream_t stream = nullptr;
    uint64_t bits = 0;
    bool poisoned = false;
};

namespace {

size_t pad2048(size_t n) { return (n + 2047) / 2048 * 2048; }

void destroy(mickey128_state *st)
{
    if (!st) return;
    if (st->stream || st->planes) (void)hipStreamSynchronize(st->stream);
    if (st->planes) (void)hipFree(st->planes);
    if (st->stage) (void)hipFree(st->stage);
    if (st->host_status) (void)hipHostFree(st->host_status);
    delete st;
}

}  // namespace

extern "C" {

mickey128_state *mickey128_init(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n,
                                void *hip_stream)
{
    if (!keys || !ivs || n == 0) {
        fail(MICKEY_EINVAL, "mickey128_init: NULL keys/ivs or n == 0");
        return nullptr;
    }
    if (n > ((size_t)1 << 31)) {
        fail(MICKEY_EINVAL, "mickey128_init: n = %zu exceeds 2^31 instances", n);
        return nullptr;
    }
    mickey128_state *st = new (std::nothrow) mickey128_state;
    if (!st) {
        fail(MICKEY_ENOMEM, "mickey128_init: host allocation failed");
        return nullptr;
    }
    st->n = n;
    st->n_pad = pad2048(n);
    st->nslices = st->n_pad / 32;
    st->stream = (hipStream_t)hip_stream;
    const size_t ns = st->nslices;
    if (hipMalloc(&st->planes, (size_t)2 * kN * ns * 4) != hipSuccess ||
        hipMalloc(&st->stage, ((size_t)(kInputPlanes + kMaskPlanes) * ns + 1) * 4) != hipSuccess ||
        hipHostMalloc(&st->host_status, 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        destroy(st);
        fail(MICKEY_ENOMEM, "mickey128_init: device allocation failed");
        return nullptr;
    }
    uint32_t *in_planes = st->stage, *mask_planes = st->stage + (size_t)kInputPlanes * ns;
    uint32_t *status = mask_planes + (size_t)kMaskPlanes * ns;
    int rc = MICKEY_OK;
    if (hipMemsetAsync(status, 0, 4, st->stream) != hipSuccess) rc = fail(MICKEY_EDEVICE, "mickey128_init: memset");
    if (rc == MICKEY_OK) {
        m128_stage_kernel<<<dim3((unsigned)(ns / 8)), dim3(256), 0, st->stream>>>(
            keys, ivs, iv_bits, (uint32_t)n, (uint32_t)ns, in_planes, mask_planes, status);
        rc = check_launch("mickey128 stage");
    }
    if (rc == MICKEY_OK && iv_bits) {
        // refuse IV lengths over 128 before any register is initialised from them
        if (hipMemcpyAsync(st->host_status, status, 4, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
            hipStreamSynchronize(st->stream) != hipSuccess)
            rc = fail(MICKEY_EDEVICE, "mickey128_init: status read-back failed");
        else if (*st->host_status)
            rc = fail(MICKEY_EINVAL, "mickey128_init: an IV length exceeds 128 bits");
    }
    if (rc == MICKEY_OK) {
        m128_init_kernel<<<dim3((unsigned)(ns / kSlicesPerGroup)), dim3(128), 0, st->stream>>>(
            in_planes, mask_planes, st->planes, (uint32_t)ns);
        rc = check_launch("mickey128 init");
    }
    if (rc != MICKEY_OK) {
        destroy(st);
        return nullptr;
    }
    ok();
    return st;
}

int mickey128_generate(mickey128_state *st, uint64_t nbits, void *out)
{
    if (!st || !out || nbits == 0) return fail(MICKEY_EINVAL, "mickey128_generate: NULL state/out or nbits == 0");
    if (st->poisoned) return fail(MICKEY_EDEVICE, "mickey128_generate: the state was poisoned by an earlier failure");
    if (st->bits + nbits < st->bits) return fail(MICKEY_ERANGE, "mickey128_generate: bit counter overflow");
    m128_gen_kernel<<<dim3((unsigned)(st->nslices / kSlicesPerGroup)), dim3(128), 0, st->stream>>>(
        st->planes, (uint32_t)st->nslices, nbits, (uint32_t *)out);
    // a launch that is refused leaves the registers as they were
    if (check_launch("mickey128 generate") != MICKEY_OK) return MICKEY_EDEVICE;
    st->bits += nbits;
    return ok();
}

int mickey128_sync(mickey128_state *st)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey128_sync: NULL state");
    if (hipStreamSynchronize(st->stream) != hipSuccess) {
        st->poisoned = true;
        return fail(MICKEY_EDEVICE, "mickey128_sync: %s", hipGetErrorString(hipGetLastError()));
    }
    return st->poisoned ? fail(MICKEY_EDEVICE, "mickey128_sync: the state is poisoned") : ok();
}

int mickey128_export(const mickey128_state *st, uint32_t *planes)
{
    if (!st || !planes) return fail(MICKEY_EINVAL, "mickey128_export: NULL argument");
    if (hipMemcpyAsync(planes, st->planes, (size_t)2 * kN * st->nslices * 4, hipMemcpyDeviceToDevice, st->stream) !=
        hipSuccess)
        return fail(MICKEY_EDEVICE, "mickey128_export: copy failed");
    return ok();
}

void mickey128_free(mickey128_state *st) { destroy(st); }

size_t mickey128_num_instances(const mickey128_state *st) { return st ? st->n : 0; }

uint64_t mickey128_bits_generated(const mickey128_state *st) { return st ? st->bits : 0; }

size_t mickey128_plane_pitch(size_t n) { return pad2048(n) / 8; }

int mickey128_ops_per_clock(void) { return ops_per_clock(); }

}  // extern "C"
