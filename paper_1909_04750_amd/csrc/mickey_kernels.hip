// HIP kernels and C-ABI of libmickey.so: bitsliced MICKEY 2.0 on MI355X (gfx950).
//
// Data layout in HBM (n_pad = 64*ceil(n/64) instances, nslices = n_pad/32):
//   state   200 planes x nslices u32: plane j < 100 is r_j, plane 100+j is s_j; bit l of
//           word g is instance 32g+l.  Planes are contiguous (pitch nslices*4 bytes).
//   input   160 planes of input bits (IV part right-aligned to clock 80, then key bits)
//           and 80 planes of "lane has started" masks, same shape; temporary.
//   output  see include/mickey.h.
// Execution: one lane owns one 32-instance slice (K=1) or two adjacent slices (K=2)
// and keeps its 200 state words in VGPRs for the whole call; one wave64 block per 64
// lanes; no LDS except the row-major transpose staging.
#include "mickey_device.h"
#include "mickey_host.h"
#include "mickey_state.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace mickey;
using namespace mickey_host;

namespace {

constexpr int kUnroll = 4;  // clocks per loop iteration of the generate kernels
constexpr int kSplitWaves = 4;   // waves per SIMD the split kernel is compiled for (128 VGPRs)
constexpr int kSplit4Waves = 4;  // ... and the four-wave split (128 VGPRs)

// ------------------------------------------------------------------------ kernels

// a2: initialisation.  One lane per slice; R = S = 0 then 260 mixing clocks, and the
// registers are stored as the state planes.
template <bool MASKED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void init_kernel(
    const uint32_t *__restrict__ in_planes, const uint32_t *__restrict__ mask_planes,
    uint32_t *__restrict__ state, uint32_t nslices)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    Regs<1> x;
    init_clocks<MASKED, kUnroll>(x, in_planes, mask_planes, pitch, voff);
    store_state<1>(x, state, pitch, voff);
}

template <int K>
struct GenOccupancy;
template <>
struct GenOccupancy<1> {
    static constexpr int waves = 2;
};
template <>
struct GenOccupancy<2> {
    static constexpr int waves = 1;
};

// a3 + a4 + a6: keystream clocks with the bit-plane store of every clock and the
// state write-back at the end.  Lane g owns words g*K*4 .. of every plane.
template <int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GenOccupancy<K>::waves,
                                                                    GenOccupancy<K>::waves))) void
gen_bitsliced_kernel(uint32_t *__restrict__ state, uint32_t ngroups, uint32_t pitch32, uint64_t nbits,
                     uint32_t *__restrict__ out)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= ngroups) return;
    const size_t pitch = (size_t)pitch32;
    const uint32_t voff = g * 4u * K;
    Regs<K> x;
    load_state<K>(x, state, pitch, voff);
    char *plane = (char *)out;  // wave-uniform
    uint64_t t = 0;
    for (; t + kUnroll <= nbits; t += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            store_plane<K>(plane, voff, x.r[0] ^ x.s[0]);
            plane += pitch;
            clock_gen<K>(x);
        }
    }
    for (; t < nbits; t++) {
        store_plane<K>(plane, voff, x.r[0] ^ x.s[0]);
        plane += pitch;
        clock_gen<K>(x);
    }
    store_state<K>(x, state, pitch, voff);
}

// a3 + a5 + a6: keystream clocks with delivery as per-instance row-major words: every
// 32 clocks each lane turns its 32 keystream words into one word per instance and
// stores it as u32 and/or exact f32 ((w >> 8) * 2^-24).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void gen_rowmajor_kernel(
    uint32_t *__restrict__ state, uint32_t nslices, uint32_t n, uint64_t nwords, uint32_t *__restrict__ out_u32,
    float *__restrict__ out_f32)
{
    __shared__ uint32_t zbuf[32][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + tid;
    if (g >= nslices) return;  // no barriers below: each lane only touches its LDS column
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    Regs<1> x;
    load_state<1>(x, state, pitch, voff);
    const uint32_t first = g * 32u;
    const uint32_t valid = n > first ? (n - first < 32u ? n - first : 32u) : 0u;
    uint32_t *ou = out_u32 ? out_u32 + (size_t)first * nwords : nullptr;
    float *of = out_f32 ? out_f32 + (size_t)first * nwords : nullptr;
    for (uint64_t j = 0; j < nwords; j++) {
        rowmajor_block<kUnroll>(x, zbuf, tid, [&](int l, uint32_t w) {
            if ((uint32_t)l < valid) {
                const size_t off = (size_t)l * nwords + j;
                if (ou) ou[off] = w;
                if (of) of[off] = (float)(w >> 8) * 0x1p-24f;
            }
        });
    }
    store_state<1>(x, state, pitch, voff);
}

// Split generate, for calls with too few slices to give every SIMD two waves: a
// workgroup of two waves serves 64 slices, wave 0 holding the R words and wave 1 the S
// words, so each clock is two half-clocks running side by side on two SIMDs.  Per
// clock the waves swap what the other register's update needs, through a
// double-buffered LDS slot and one barrier: R sends r_33 (for c_S), S sends s_34 (for
// c_R) and s_0 (for the keystream bit z = r_0 ^ s_0, which the R wave forms and
// delivers).  Each wave writes its value as soon as its own update has made it final
// (R after r_99..r_33, S after s_1..s_34) and reads the other's after the barrier, so
// the LDS round trip overlaps the rest of its half-clock.  The buffer a clock writes
// is the one the clock after next reads again, so one barrier per clock suffices.
// ROWMAJOR: 32-clock blocks staged in LDS and transposed as in gen_rowmajor_kernel
// (nbits % 32 == 0); otherwise one bit-plane word per clock as in gen_bitsliced_kernel.
template <bool ROWMAJOR>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(kSplitWaves, kSplitWaves))) void
gen_split_kernel(uint32_t *__restrict__ state, uint32_t nslices, uint32_t n, uint64_t nbits,
                 uint32_t *__restrict__ out, uint32_t *__restrict__ out_u32, float *__restrict__ out_f32)
{
    __shared__ SplitLds xl;
    __shared__ uint32_t zbuf[ROWMAJOR ? 32 : 1][64];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const uint32_t g = blockIdx.x * 64u + lane;
    // Lanes past the last slice run a copy of the block's first slice (g0 < nslices):
    // every word they store equals the one that slice's own lane stores at the same
    // address in the same instruction, so no store needs a branch.
    const uint32_t gs = g < nslices ? g : blockIdx.x * 64u;
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = gs * 4u;
    Regs<1> x;
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < 100; j++) x.r[j] = ld_word<1>((const char *)state + (size_t)j * pitch + voff);
        xl.r33[0][lane] = x.r[kRCut].w[0];
        lds_barrier();
        Word<1> s34 = {{xl.s34[0][lane]}}, s0 = {{xl.s0[0][lane]}};
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (ROWMAJOR) {
            const uint64_t nwords = nbits / 32;
            const uint32_t first = g * 32u;
            const uint32_t valid = n > first ? (n - first < 32u ? n - first : 32u) : 0u;
            uint32_t *ou = out_u32 ? out_u32 + (size_t)first * nwords : nullptr;
            float *of = out_f32 ? out_f32 + (size_t)first * nwords : nullptr;
            for (uint64_t j = 0; j < nwords; j++) {
                for (int b0 = 0; b0 < 32; b0 += kUnroll) {
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        zbuf[31 - (b0 + u)][lane] = (x.r[0] ^ s0).w[0];  // row 31-b holds clock b
                        split_r_clock(x, s34, s0, xl, lane, (u + 1) & 1);
                    }
                }
                rowmajor_flush(zbuf, lane, [&](int l, uint32_t w) {
                    if ((uint32_t)l < valid) {
                        const size_t off = (size_t)l * nwords + j;
                        if (ou) store_global(ou + off, w);
                        if (of) store_global_f32(of + off, (float)(w >> 8) * 0x1p-24f);
                    }
                });
            }
        } else {
            char *plane = (char *)out;  // wave-uniform
            uint64_t t = 0;
            for (; t + kUnroll <= nbits; t += kUnroll) {
#pragma unroll
                for (int u = 0; u < kUnroll; u++) {
                    store_plane<1>(plane, voff, x.r[0] ^ s0);
                    plane += pitch;
                    split_r_clock(x, s34, s0, xl, lane, (u + 1) & 1);
                }
            }
            for (; t < nbits; t++) {
                store_plane<1>(plane, voff, x.r[0] ^ s0);
                plane += pitch;
                split_r_clock(x, s34, s0, xl, lane, (int)((t + 1) & 1));
            }
        }
        uint32_t v = voff;
        asm volatile("" : "+v"(v));  // keep the load addresses from living across the loop
#pragma unroll
        for (int j = 0; j < 100; j++) st_word<1>((char *)state + (size_t)j * pitch + v, x.r[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 100; j++) x.s[j] = ld_word<1>((const char *)state + (size_t)(100 + j) * pitch + voff);
        xl.s34[0][lane] = x.s[kSCut].w[0];
        xl.s0[0][lane] = x.s[0].w[0];
        lds_barrier();
        Word<1> r33 = {{xl.r33[0][lane]}};
        __builtin_amdgcn_sched_barrier(0);
        // the same clock count and buffer sequence as the R wave (one barrier per clock);
        // ascending and descending sweeps alternate, so the S words keep one register set
        static_assert(kUnroll % 2 == 0, "sweeps alternate in pairs");
        uint64_t t = 0;
        for (; t + kUnroll <= nbits; t += kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; u += 2) {
                split_s_clock(x, r33, xl, lane, 1);
                split_s_clock_desc(x, r33, xl, lane, 0);
            }
        }
        // at most kUnroll - 1 = 3 clocks left, starting on an even clock (straight-line, so
        // the registers need not return to their loop positions)
        if (t < nbits) split_s_clock(x, r33, xl, lane, 1);
        if (t + 1 < nbits) split_s_clock_desc(x, r33, xl, lane, 0);
        if (t + 2 < nbits) split_s_clock(x, r33, xl, lane, 1);
        uint32_t v = voff;
        asm volatile("" : "+v"(v));
#pragma unroll
        for (int j = 0; j < 100; j++) st_word<1>((char *)state + (size_t)(100 + j) * pitch + v, x.s[j]);
    }
}

// Four-wave split (the clock of mickey_device.h: halves of R and S on four waves), for
// launches that the two-wave split still leaves at one wave per SIMD.  ~75-92 VALU per
// wave per clock.
// One wave's part of gen_split4_kernel (ROLE = wave index); every role passes 1 + nbits
// barriers.
template <int ROLE>
__device__ __forceinline__ void s4_run(uint32_t *__restrict__ state, size_t pitch, uint32_t voff, uint64_t nbits,
                                       uint32_t *__restrict__ out, Split4Lds &xl, uint32_t lane)
{
    constexpr bool kR = ROLE < 2;
    constexpr int j0 = ROLE == 0 || ROLE == 2 ? 0 : 50;  // first position of the half
    constexpr int base = kR ? 0 : 100;                  // r or s planes
    Regs<1> x;
    S4In in;
#pragma unroll
    for (int j = 0; j < 50; j++) {
        const Word<1> v = ld_word<1>((const char *)state + (size_t)(base + j0 + j) * pitch + voff);
        if constexpr (kR) x.r[j0 + j] = v;
        else x.s[j0 + j] = v;
    }
    // publish the state-0 exchange values, then read the others'
    if constexpr (ROLE == 0) {
        xl.v[0][kX_R49][lane] = x.r[49].w[0];
        xl.v[0][kX_R33][lane] = x.r[33].w[0];
    } else if constexpr (ROLE == 1) {
        xl.v[0][kX_R99][lane] = x.r[99].w[0];
        xl.v[0][kX_R67][lane] = x.r[67].w[0];
    } else if constexpr (ROLE == 2) {
        xl.v[0][kX_S49][lane] = x.s[49].w[0];
        xl.v[0][kX_S34][lane] = x.s[34].w[0];
        xl.v[0][kX_S0][lane] = x.s[0].w[0];
    } else {
        xl.v[0][kX_S50][lane] = x.s[50].w[0];
        xl.v[0][kX_S99][lane] = x.s[99].w[0];
        xl.v[0][kX_S67][lane] = x.s[67].w[0];
    }
    lds_barrier();
    if constexpr (ROLE == 0) {
        in.a.w[0] = xl.v[0][kX_R99][lane];
        in.b.w[0] = xl.v[0][kX_R67][lane];
        in.c.w[0] = xl.v[0][kX_S34][lane];
        in.d.w[0] = xl.v[0][kX_S0][lane];
    } else if constexpr (ROLE == 1) {
        x.r[49].w[0] = xl.v[0][kX_R49][lane];
        in.a.w[0] = xl.v[0][kX_S34][lane];
    } else if constexpr (ROLE == 2) {
        x.s[50].w[0] = xl.v[0][kX_S50][lane];
        in.a.w[0] = xl.v[0][kX_S99][lane];
        in.b.w[0] = xl.v[0][kX_S67][lane];
        in.c.w[0] = xl.v[0][kX_R33][lane];
    } else {
        x.s[49].w[0] = xl.v[0][kX_S49][lane];
        in.a.w[0] = xl.v[0][kX_R33][lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    auto clock = [&](auto ph) {
        constexpr int PH = decltype(ph)::value;
        if constexpr (ROLE == 0) s4_clock_rlo<PH>(x, in, xl, lane);
        else if constexpr (ROLE == 1) s4_clock_rhi<PH>(x, in, xl, lane);
        else if constexpr (ROLE == 2) s4_clock_slo<PH>(x, in, xl, lane);
        else s4_clock_shi<PH>(x, in, xl, lane);
    };
    // clock t writes buffer (t + 1) & 1: two clocks per iteration keep the buffer index (and
    // the register sets of the functional update) fixed; an odd last clock writes buffer 1
    char *plane = (char *)out;  // wave-uniform (used by wave 0)
    const uint64_t npairs = nbits / 2;
    for (uint64_t i = 0; i < npairs; i++) {
        if constexpr (ROLE == 0) {
            store_plane<1>(plane, voff, x.r[0] ^ in.d);
            plane += pitch;
        }
        clock(std::integral_constant<int, 1>{});
        if constexpr (ROLE == 0) {
            store_plane<1>(plane, voff, x.r[0] ^ in.d);
            plane += pitch;
        }
        clock(std::integral_constant<int, 0>{});
    }
    if (nbits & 1) {
        if constexpr (ROLE == 0) store_plane<1>(plane, voff, x.r[0] ^ in.d);
        clock(std::integral_constant<int, 1>{});
    }
    uint32_t v = voff;
    asm volatile("" : "+v"(v));  // keep the load addresses from living across the loop
#pragma unroll
    for (int j = 0; j < 50; j++) {
        if constexpr (kR) st_word<1>((char *)state + (size_t)(base + j0 + j) * pitch + v, x.r[j0 + j]);
        else st_word<1>((char *)state + (size_t)(base + j0 + j) * pitch + v, x.s[j0 + j]);
    }
}

// Bit-plane output only (the row-major layouts reach it through the staged transpose).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kSplit4Waves, kSplit4Waves))) void
gen_split4_kernel(uint32_t *__restrict__ state, uint32_t nslices, uint64_t nbits, uint32_t *__restrict__ out)
{
    __shared__ Split4Lds xl;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * 64u + lane;
    // lanes past the last slice run a copy of the block's first slice (see gen_split_kernel)
    const uint32_t gs = g < nslices ? g : blockIdx.x * 64u;
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = gs * 4u;
    if (wave == 0) s4_run<0>(state, pitch, voff, nbits, out, xl, lane);
    else if (wave == 1) s4_run<1>(state, pitch, voff, nbits, out, xl, lane);
    else if (wave == 2) s4_run<2>(state, pitch, voff, nbits, out, xl, lane);
    else s4_run<3>(state, pitch, voff, nbits, out, xl, lane);
}

// a5, staged: a chunk of bit-planes (as the generate kernels write them) turned into
// row-major words by the tiled transpose of tile_to_rows, so that every row segment goes
// out as whole 128-byte lines.  The fused delivery above stores one 4-byte word per
// instance every 32 clocks, i.e. 64 lines per store instruction, which the memory system
// serves at about 0.3 TB/s; here each store instruction writes two lines.
__global__ __launch_bounds__(256) void rowmajor_transpose_kernel(const uint32_t *__restrict__ planes,
                                                                 uint32_t nslices, uint32_t nclocks, uint32_t n,
                                                                 uint64_t nwords, uint64_t w0,
                                                                 uint32_t *__restrict__ out_u32,
                                                                 float *__restrict__ out_f32)
{
    __shared__ uint32_t lds[kTpLdsWords];
    const uint32_t tid = threadIdx.x;
    const uint2 tb = tile_of_block();
    const uint32_t s0 = tb.x * kTpSlices;
    const uint32_t t0 = tb.y * kTpClocks;
    const uint32_t nb = min((uint32_t)kTpBlocks, (nclocks - t0) / 32u);  // blocks in this tile
    tile_to_rows(lds, planes, nslices, s0, t0, nb, tid, [] {});
    const uint32_t w = tid & 31u;
    if (w < nb) {
        for (uint32_t i = tid >> 5; i < 32u * kTpSlices; i += 8u) {
            const uint32_t inst = 32u * s0 + i;
            if (inst >= n) break;
            const uint32_t v = tile_row_word(lds, i, w);
            const size_t off = (size_t)inst * nwords + w0 + t0 / 32u + w;
            if (out_u32) store_global(out_u32 + off, v);
            if (out_f32) store_global_f32(out_f32 + off, (float)(v >> 8) * 0x1p-24f);
        }
    }
}

// State export: one thread per instance packs its 200 bits (r_0..r_99, s_0..s_99)
// MSB first into 25 bytes.
__global__ __launch_bounds__(256) void export_kernel(const uint32_t *__restrict__ state, uint32_t nslices,
                                                     uint32_t n, uint8_t *__restrict__ packed)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t g = i >> 5, l = i & 31u;
    uint8_t *dst = packed + 25ull * i;
    for (int byte = 0; byte < 25; byte++) {
        uint32_t v = 0;
        for (int k = 0; k < 8; k++) {
            const int j = byte * 8 + k;
            v = (v << 1) | ((state[(size_t)j * nslices + g] >> l) & 1u);
        }
        dst[byte] = (uint8_t)v;
    }
}

// State import: one thread per instance (n_pad threads); ballots rebuild the plane
// words, pad lanes keep their old bits.
__global__ __launch_bounds__(256) void import_kernel(const uint8_t *__restrict__ packed, uint32_t n,
                                                     uint32_t nslices, uint32_t *__restrict__ state)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslices * 32u) return;  // whole waves only (n_pad is a multiple of 64)
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t word = i >> 5;
    const bool have = i < n;
    const uint64_t vm = __ballot(have);
    const uint32_t vmask = (lane < 32u) ? (uint32_t)vm : (uint32_t)(vm >> 32);
    for (int j = 0; j < 200; j++) {
        const uint32_t bit = have ? ((packed[25ull * i + (j >> 3)] >> (7 - (j & 7))) & 1u) : 0u;
        const uint64_t bal = __ballot(bit);
        if (lane == 0u || lane == 32u) {
            const uint32_t nw = (lane == 0u) ? (uint32_t)bal : (uint32_t)(bal >> 32);
            uint32_t *p = state + (size_t)j * nslices + word;
            *p = (*p & ~vmask) | (nw & vmask);
        }
    }
}

}  // namespace

// ------------------------------------------------------------------------ C ABI

// Scratch of the allocation-free entry point (mickey_generate_rowmajor_noalloc): the staged
// path's register snapshot and its two bit-plane chunk buffers.  Every device that runs the
// library holds one copy until the process ends; nothing in it has to start at zero (each
// call writes what it later reads).  Host code reaches it only through the per-device
// address from hipGetSymbolAddress, never through the array's name.
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / 4];

namespace mickey_host {

thread_local int g_err = MICKEY_OK;
thread_local char g_msg[256] = "";

int fail(int code, const char *fmt, ...)
{
    g_err = code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

int ok()
{
    g_err = MICKEY_OK;
    g_msg[0] = 0;
    return MICKEY_OK;
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return MICKEY_OK;
}

void prefix_error(const char *prefix)
{
    char msg[sizeof g_msg];
    memcpy(msg, g_msg, sizeof msg);
    snprintf(g_msg, sizeof g_msg, "%s: %s", prefix, msg);
}

// Device address of `scratch` on each device, taken once per device with that device
// current (the first mickey_init on it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_addr[kMaxDevices] = {};

int scratch_address(int device, uint32_t **addr)
{
    if (device < 0 || device >= kMaxDevices) return fail(MICKEY_EDEVICE, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MICKEY_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch_addr[device] = (uint32_t *)p;
    }
    *addr = g_scratch_addr[device];
    return MICKEY_OK;
}

// Launches left before an injected failure (0: none pending); see mickey_debug_fail_launch.
std::atomic<int> g_fail_in{0};

int launch_guard(const char *what)
{
    int k = g_fail_in.load();
    while (k > 0 && !g_fail_in.compare_exchange_weak(k, k - 1)) {
    }
    if (k == 1) return fail(MICKEY_EDEVICE, "%s: injected launch failure", what);
    return MICKEY_OK;
}

int ensure_side(mickey_state *st)
{
    if (st->side) return MICKEY_OK;
    bool okc = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking) == hipSuccess;
    for (int b = 0; b < 2 && okc; b++)
        okc = hipEventCreateWithFlags(&st->ev_gen[b], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&st->ev_tp[b], hipEventDisableTiming) == hipSuccess;
    okc = okc && hipEventCreateWithFlags(&st->ev_fork, hipEventDisableTiming) == hipSuccess &&
          hipEventCreateWithFlags(&st->ev_join, hipEventDisableTiming) == hipSuccess;
    if (!okc) {
        (void)hipGetLastError();
        return fail(MICKEY_EDEVICE, "cannot create the state's second stream or its events");
    }
    return MICKEY_OK;
}

int ensure_scratch(mickey_state *st, size_t bytes)
{
    if (st->bmem_bytes >= bytes) return MICKEY_OK;
    if (st->bmem) {  // work queued earlier may still read it
        (void)hipStreamSynchronize(st->stream);
        if (st->side) (void)hipStreamSynchronize(st->side);
        (void)hipFree(st->bmem);
        st->bmem = nullptr;
        st->bmem_bytes = 0;
    }
    const size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (hipMalloc(&st->bmem, want) != hipSuccess) {
        (void)hipGetLastError();
        st->bmem = nullptr;
        return fail(MICKEY_ENOMEM, "cannot allocate %zu bytes of scratch", want);
    }
    st->bmem_bytes = want;
    return MICKEY_OK;
}

}  // namespace mickey_host

namespace {

// Largest instance count the 32-bit indexing of the kernels supports.
constexpr size_t kMaxInstances = (size_t)1 << 31;

// a1 + a2 on an allocated state: stage the inputs, run the 260 initialisation clocks,
// reset the bit counters.  With iv_bits the lengths are validated (stream sync) after the
// staging and before the initialisation touches the registers, so a refused length leaves
// the state as it was.
int run_init(mickey_state *st, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits)
{
    if (!keys || !ivs) return fail(MICKEY_EINVAL, "keys and ivs must be device pointers");
    uint32_t *in_planes = st->stage;
    uint32_t *mask_planes = st->stage + (size_t)kInputPlanes * st->nslices;
    uint32_t *status = mask_planes + (size_t)kMaskPlanes * st->nslices;
    if (hipMemsetAsync(status, 0, 4, st->stream) != hipSuccess) return check_launch("hipMemsetAsync");
    const dim3 sgrid((unsigned)((st->n_pad + 255) / 256));
    int rc = launch_guard("stage_kernel");
    if (rc != MICKEY_OK) return rc;
    if (iv_bits)
        hipLaunchKernelGGL((stage_kernel<true, false>), sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits,
                           nullptr, (uint32_t)st->n, (uint32_t)st->nslices, in_planes, mask_planes, status);
    else
        hipLaunchKernelGGL((stage_kernel<false, false>), sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits,
                           nullptr, (uint32_t)st->n, (uint32_t)st->nslices, in_planes, mask_planes, status);
    rc = check_launch("stage_kernel");
    if (rc != MICKEY_OK) return rc;
    if (iv_bits) {
        if (hipMemcpyAsync(st->host_status, status, 4, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
            hipStreamSynchronize(st->stream) != hipSuccess)
            return check_launch("IV length check");
        if (*st->host_status) return fail(MICKEY_EINVAL, "an IV length exceeds 80 bits");
    }
    rc = launch_guard("init_kernel");
    if (rc != MICKEY_OK) return rc;
    const dim3 grid((unsigned)((st->nslices + 63) / 64));
    if (iv_bits)
        hipLaunchKernelGGL(init_kernel<true>, grid, dim3(64), 0, st->stream, in_planes, mask_planes, st->planes,
                           (uint32_t)st->nslices);
    else
        hipLaunchKernelGGL(init_kernel<false>, grid, dim3(64), 0, st->stream, in_planes, mask_planes, st->planes,
                           (uint32_t)st->nslices);
    rc = check_launch("init_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits = 0;
    st->extra.clear();
    st->max_extra = 0;
    st->snap_valid = false;
    st->poisoned = false;
    return MICKEY_OK;
}

void destroy(mickey_state *st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->stream);
    if (st->side) (void)hipStreamSynchronize(st->side);
    if (st->planes) (void)hipFree(st->planes);
    if (st->stage) (void)hipFree(st->stage);
    if (st->host_status) (void)hipHostFree(st->host_status);
    if (st->chunk) (void)hipFree(st->chunk);
    if (st->snap) (void)hipFree(st->snap);
    if (st->bmem) (void)hipFree(st->bmem);
    if (st->bhost_ev) (void)hipEventSynchronize(st->bhost_ev);
    if (st->bhost) (void)hipHostFree(st->bhost);
    hipEvent_t evs[] = {st->ev_gen[0], st->ev_gen[1], st->ev_tp[0], st->ev_tp[1], st->bhost_ev, st->ev_fork,
                        st->ev_join};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    if (st->side) (void)hipStreamDestroy(st->side);
    delete st;
}

mickey_state *init_impl(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n,
                        hipStream_t stream)
{
    if (!keys || !ivs) {
        fail(MICKEY_EINVAL, "mickey_init: keys and ivs must be device pointers");
        return nullptr;
    }
    if (n == 0 || n > kMaxInstances) {
        fail(MICKEY_EINVAL, "mickey_init: n must be in 1..2^31 (got %zu)", n);
        return nullptr;
    }
    mickey_state *st = new (std::nothrow) mickey_state();
    if (!st) {
        fail(MICKEY_ENOMEM, "mickey_init: host allocation failed");
        return nullptr;
    }
    st->n = n;
    st->n_pad = pad64(n);
    st->nslices = st->n_pad / 32;
    st->stream = stream;
    st->word_bits = 32;
    st->schedule = MICKEY_SCHED_AUTO;
    st->transpose = MICKEY_TRANSPOSE_AUTO;
    (void)hipGetDevice(&st->device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, st->device) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    st->simds = 4 * cus;
    const size_t pitch = st->nslices * 4;
    const size_t stage_bytes = (size_t)(kInputPlanes + kMaskPlanes) * pitch + 256;
    if (hipMalloc(&st->planes, 200 * pitch) != hipSuccess || hipMalloc(&st->stage, stage_bytes) != hipSuccess ||
        hipHostMalloc((void **)&st->host_status, 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        destroy(st);
        fail(MICKEY_ENOMEM, "mickey_init: cannot allocate %zu bytes of device memory", 200 * pitch + stage_bytes);
        return nullptr;
    }
    int rc = run_init(st, keys, ivs, iv_bits);
    if (rc == MICKEY_OK) rc = scratch_address(st->device, &st->noalloc);
    if (rc != MICKEY_OK) {
        destroy(st);
        prefix_error("mickey_init");
        return nullptr;
    }
    ok();
    return st;
}

// Which kernel generates: the split schedules multiply the waves of a call by 2 or 4 at the
// cost of a per-clock exchange.  Measured on MI355X (1024 SIMDs, bit-planes, 8192 clocks;
// ms): at 2^22 instances one-wave 6.95, two-wave split 7.50, four-wave split 7.76 (the
// one-wave kernel fills every SIMD with two waves); at 2^21 5.00, 3.84, 4.05 (the two-wave
// split, at 128 VGPRs, puts two waves on every SIMD); at 2^20 5.08, 3.49, 2.20.  The
// automatic schedule follows: one-wave from two one-wave waves per SIMD, the two-wave
// split from one, the four-wave split below.
enum class Gen { OneWave, Split2, Split4 };

Gen pick_gen(const mickey_state *st)
{
    if (st->word_bits != 32 || st->schedule == MICKEY_SCHED_ONE_WAVE) return Gen::OneWave;
    if (st->schedule == MICKEY_SCHED_SPLIT) return Gen::Split2;
    if (st->schedule == MICKEY_SCHED_SPLIT4) return Gen::Split4;
    const size_t waves = (st->nslices + 63) / 64;
    if (waves >= 2 * (size_t)st->simds) return Gen::OneWave;
    return waves >= (size_t)st->simds ? Gen::Split2 : Gen::Split4;
}

bool use_split4(const mickey_state *st) { return pick_gen(st) == Gen::Split4; }

// The fused row-major path has one-wave and two-wave kernels; the four-wave schedule
// uses the two-wave one there.
bool use_split(const mickey_state *st) { return pick_gen(st) != Gen::OneWave; }

// Staged row-major delivery: clocks per chunk for chunk buffers of at most 512 MiB each, in
// whole transpose tiles (1024 clocks) and at most 8192; 0 when even one tile of planes
// would exceed 2 GiB (the fused path then serves MICKEY_TRANSPOSE_AUTO).
uint64_t staged_chunk_clocks(const mickey_state *st)
{
    const uint64_t pitch = st->nslices * 4;
    if ((uint64_t)kTpClocks * pitch > (2ull << 30)) return 0;
    uint64_t c = ((512ull << 20) / pitch) / kTpClocks * kTpClocks;
    if (c < (uint64_t)kTpClocks) c = kTpClocks;
    if (c > 8192) c = 8192;
    return c;
}

int launch_generate_planes(mickey_state *st, uint64_t nbits, uint32_t *out);

// Chunk k is generated on the state's stream into buffer k % 2 and transposed on the
// side stream, so the transpose of chunk k (HBM-bound) overlaps the generation of chunk
// k + 1 (VALU-bound) where the generate kernel leaves room on the CUs.  Events order each
// transpose after its chunk, each chunk after the transpose that last read its buffer,
// and the state's stream after the last transpose.  Measured on MI355X at 2^20
// instances, the overlap pays beside the two-wave split (1.87 ms per 4096-clock chunk
// instead of 2.07 serially) but not beside the four-wave split, whose waves and the
// transpose's slow each other down more than they overlap (2.0 ms instead of 1.8): with
// that schedule the transposes run on the state's stream.
// The registers are first copied to `snap` (200 planes): if a launch after the first
// generate fails, they are copied back, so the call fails with the state unchanged; if
// even that copy cannot be enqueued, the state is poisoned.
//   chunk: two buffers of chunk_clocks planes each (chunk_clocks a multiple of 32)
//   overlap: transposes may run on the side stream (else everything stays on the state's
//            stream, in order, with no event)
int generate_staged_with(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32, uint32_t *chunk,
                         uint64_t chunk_clocks, uint32_t *snap, bool overlap)
{
    const size_t pitch = st->nslices * 4;
    overlap = overlap && !use_split4(st);
    int rc = overlap ? ensure_side(st) : MICKEY_OK;
    if (rc != MICKEY_OK) return rc;
    rc = launch_guard("state snapshot");
    if (rc != MICKEY_OK) return rc;
    if (hipMemcpyAsync(snap, st->planes, 200 * pitch, hipMemcpyDeviceToDevice, st->stream) != hipSuccess)
        return check_launch("state snapshot");
    const uint64_t nwords = nbits / 32;
    hipStream_t tp_stream = overlap ? st->side : st->stream;
    int last = 0;
    uint64_t k = 0;
    bool changed = false;  // a generate kernel has been launched on the registers
    for (uint64_t c0 = 0; c0 < nbits && rc == MICKEY_OK; c0 += chunk_clocks, k++) {
        const int b = (int)(k & 1);
        uint32_t *buf = chunk + (size_t)b * chunk_clocks * st->nslices;
        const uint64_t nc = nbits - c0 < chunk_clocks ? nbits - c0 : chunk_clocks;
        if (overlap && k >= 2 && hipStreamWaitEvent(st->stream, st->ev_tp[b], 0) != hipSuccess) {
            rc = check_launch("hipStreamWaitEvent");
            break;
        }
        rc = launch_generate_planes(st, nc, buf);
        if (rc != MICKEY_OK) break;
        changed = true;
        if (overlap && (hipEventRecord(st->ev_gen[b], st->stream) != hipSuccess ||
                        hipStreamWaitEvent(tp_stream, st->ev_gen[b], 0) != hipSuccess)) {
            rc = check_launch("hipEventRecord");
            break;
        }
        rc = launch_guard("rowmajor_transpose_kernel");
        if (rc != MICKEY_OK) break;
        const dim3 grid((unsigned)((st->nslices + kTpSlices - 1) / kTpSlices),
                        (unsigned)((nc + kTpClocks - 1) / kTpClocks));
        hipLaunchKernelGGL(rowmajor_transpose_kernel, grid, dim3(256), 0, tp_stream, buf, (uint32_t)st->nslices,
                           (uint32_t)nc, (uint32_t)st->n, nwords, c0 / 32, out_u32, out_f32);
        rc = check_launch("rowmajor_transpose_kernel");
        if (rc != MICKEY_OK) break;
        if (overlap && hipEventRecord(st->ev_tp[b], tp_stream) != hipSuccess) {
            rc = check_launch("hipEventRecord");
            break;
        }
        last = b;
    }
    if (overlap && rc == MICKEY_OK && hipStreamWaitEvent(st->stream, st->ev_tp[last], 0) != hipSuccess)
        rc = check_launch("hipStreamWaitEvent");
    if (rc != MICKEY_OK && changed) {
        // the generate kernels all ran on the state's stream: the copy back follows them
        if (hipMemcpyAsync(st->planes, snap, 200 * pitch, hipMemcpyDeviceToDevice, st->stream) != hipSuccess) {
            (void)hipGetLastError();
            st->poisoned = true;
            st->snap_valid = snap == st->snap;
        }
    }
    return rc;
}

// The state's own chunk buffers (allocated on first use, two of `want` clocks) and snapshot.
int generate_staged(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32, uint64_t cc)
{
    const size_t pitch = st->nslices * 4;
    const uint64_t want = nbits < cc ? (nbits + kTpClocks - 1) / kTpClocks * kTpClocks : cc;
    if (st->chunk_clocks < want) {
        if (st->chunk) {
            (void)hipStreamSynchronize(st->stream);
            if (st->side) (void)hipStreamSynchronize(st->side);
            (void)hipFree(st->chunk);
            st->chunk = nullptr;
            st->chunk_clocks = 0;
        }
        if (hipMalloc(&st->chunk, 2 * want * pitch) != hipSuccess) {
            (void)hipGetLastError();
            st->chunk = nullptr;
            return fail(MICKEY_ENOMEM, "mickey_generate: cannot allocate the %llu-byte row-major chunk buffers",
                        (unsigned long long)(2 * want * pitch));
        }
        st->chunk_clocks = want;
    }
    if (!st->snap && hipMalloc(&st->snap, 200 * pitch) != hipSuccess) {
        (void)hipGetLastError();
        st->snap = nullptr;
        return fail(MICKEY_ENOMEM, "mickey_generate: cannot allocate the %zu-byte state snapshot", 200 * pitch);
    }
    return generate_staged_with(st, nbits, out_u32, out_f32, st->chunk, st->chunk_clocks, st->snap, true);
}

// nbits clocks of every instance as bit-planes (pitch nslices*4 bytes) to out.
int launch_generate_planes(mickey_state *st, uint64_t nbits, uint32_t *out)
{
    int rc = launch_guard("gen_bitsliced_kernel");
    if (rc != MICKEY_OK) return rc;
    const size_t pitch = st->nslices * 4;
    const unsigned nblocks = (unsigned)((st->nslices + 63) / 64);
    if (use_split4(st)) {
        hipLaunchKernelGGL(gen_split4_kernel, dim3(nblocks), dim3(256), 0, st->stream, st->planes,
                           (uint32_t)st->nslices, nbits, out);
    } else if (use_split(st)) {
        hipLaunchKernelGGL(gen_split_kernel<false>, dim3(nblocks), dim3(128), 0, st->stream, st->planes,
                           (uint32_t)st->nslices, (uint32_t)st->n, nbits, out, nullptr, nullptr);
    } else if (st->word_bits == 32) {
        hipLaunchKernelGGL(gen_bitsliced_kernel<1>, dim3(nblocks), dim3(64), 0, st->stream, st->planes,
                           (uint32_t)st->nslices, (uint32_t)pitch, nbits, out);
    } else {
        const size_t ngroups = st->nslices / 2;
        hipLaunchKernelGGL(gen_bitsliced_kernel<2>, dim3((unsigned)((ngroups + 63) / 64)), dim3(64), 0,
                           st->stream, st->planes, (uint32_t)ngroups, (uint32_t)pitch, nbits, out);
    }
    return check_launch("gen_bitsliced_kernel");
}

// Argument and range checks of a whole-state generate (nothing is changed).
int check_generate(const mickey_state *st, uint64_t nbits, int layout)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_generate: NULL state");
    if (st->poisoned) return fail(MICKEY_EDEVICE, "mickey_generate: the state was lost to an earlier device failure");
    if (nbits == 0) return fail(MICKEY_EINVAL, "mickey_generate: nbits must be >= 1");
    if (nbits > MICKEY_MAX_BITS_PER_IV || st->bits + st->max_extra > MICKEY_MAX_BITS_PER_IV - nbits)
        return fail(MICKEY_ERANGE, "mickey_generate: %llu + %llu bits exceeds 2^40 per key/IV pair",
                    (unsigned long long)(st->bits + st->max_extra), (unsigned long long)nbits);
    if (layout != MICKEY_BITSLICED && nbits % 32 != 0)
        return fail(MICKEY_EINVAL, "row-major layouts need nbits %% 32 == 0");
    return MICKEY_OK;
}

int generate_impl(mickey_state *st, uint64_t nbits, int layout, void *out, uint32_t *out_u32, float *out_f32)
{
    int rc = check_generate(st, nbits, layout);
    if (rc != MICKEY_OK) return rc;
    const bool split = use_split(st);
    const unsigned nblocks = (unsigned)((st->nslices + 63) / 64);
    if (layout == MICKEY_BITSLICED) {
        if (!out) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        rc = launch_generate_planes(st, nbits, (uint32_t *)out);
        if (rc != MICKEY_OK) return rc;
    } else {
        if (!out_u32 && !out_f32) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        const uint64_t cc = staged_chunk_clocks(st);
        if (st->transpose == MICKEY_TRANSPOSE_STAGED || (st->transpose == MICKEY_TRANSPOSE_AUTO && cc)) {
            rc = generate_staged(st, nbits, out_u32, out_f32, cc ? cc : (uint64_t)kTpClocks);
            if (rc != MICKEY_OK) return rc;
            st->bits += nbits;
            st->snap_valid = false;
            return ok();
        }
        rc = launch_guard("gen_rowmajor_kernel");
        if (rc != MICKEY_OK) return rc;
        if (split) {
            hipLaunchKernelGGL(gen_split_kernel<true>, dim3(nblocks), dim3(128), 0, st->stream, st->planes,
                               (uint32_t)st->nslices, (uint32_t)st->n, nbits, nullptr, out_u32, out_f32);
        } else {
            hipLaunchKernelGGL(gen_rowmajor_kernel, dim3(nblocks), dim3(64), 0, st->stream, st->planes,
                               (uint32_t)st->nslices, (uint32_t)st->n, nbits / 32, out_u32, out_f32);
        }
        rc = check_launch("gen_rowmajor_kernel");
        if (rc != MICKEY_OK) return rc;
    }
    st->bits += nbits;
    st->snap_valid = false;
    return ok();
}

// Host form of the state (mickey_state_export_host): a 32-byte header, the packed
// registers of every instance, then every instance's bit counter.
constexpr char kHostMagic[8] = {'M', 'I', 'C', 'K', 'E', 'Y', '2', 0};
constexpr uint32_t kHostVersion = 1;
struct HostHeader {
    char magic[8];
    uint32_t version;
    uint32_t state_bytes;
    uint64_t n;
    uint64_t reserved;
};
static_assert(sizeof(HostHeader) == 32, "host state header is 32 bytes");

size_t host_state_bytes(size_t n) { return sizeof(HostHeader) + n * (25 + 8); }

}  // namespace

extern "C" {

mickey_state *mickey_init(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n)
{
    return init_impl(keys, ivs, iv_bits, n, nullptr);
}

mickey_state *mickey_init_on_stream(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n,
                                    void *hip_stream)
{
    return init_impl(keys, ivs, iv_bits, n, (hipStream_t)hip_stream);
}

int mickey_generate(mickey_state *st, uint64_t nbits, void *out, int layout)
{
    switch (layout) {
    case MICKEY_BITSLICED:
        return generate_impl(st, nbits, layout, out, nullptr, nullptr);
    case MICKEY_ROWMAJOR_U32:
        if (!out) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        return generate_impl(st, nbits, layout, nullptr, (uint32_t *)out, nullptr);
    case MICKEY_ROWMAJOR_F32:
        if (!out) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        return generate_impl(st, nbits, layout, nullptr, nullptr, (float *)out);
    default:
        return fail(MICKEY_EINVAL, "mickey_generate: unknown layout %d", layout);
    }
}

int mickey_generate_rowmajor(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32)
{
    return generate_impl(st, nbits, MICKEY_ROWMAJOR_U32, nullptr, out_u32, out_f32);
}

int mickey_generate_rowmajor_noalloc(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32)
{
    int rc = check_generate(st, nbits, MICKEY_ROWMAJOR_U32);
    if (rc != MICKEY_OK) return rc;
    if (!out_u32 && !out_f32) return fail(MICKEY_EINVAL, "mickey_generate_rowmajor_noalloc: NULL output");
    const size_t pitch = st->nslices * 4;
    const size_t snap_bytes = (200 * pitch + 255) / 256 * 256;
    if (snap_bytes + 2 * 32 * pitch > kNoAllocScratchBytes)
        return fail(MICKEY_EINVAL, "mickey_generate_rowmajor_noalloc: %zu instances exceed the %zu MiB scratch "
                    "(at most %zu)", st->n, kNoAllocScratchBytes >> 20, kNoAllocScratchBytes / 264 / 4 * 32);
    uint64_t cc = (kNoAllocScratchBytes - snap_bytes) / (2 * pitch);
    cc = cc >= (uint64_t)kTpClocks ? cc / kTpClocks * kTpClocks : cc / 32 * 32;
    if (cc > 8192) cc = 8192;
    uint32_t *snap = st->noalloc;
    rc = generate_staged_with(st, nbits, out_u32, out_f32, st->noalloc + snap_bytes / 4, cc, snap, false);
    if (rc != MICKEY_OK) return rc;
    st->bits += nbits;
    st->snap_valid = false;
    return ok();
}

int mickey_rekey(mickey_state *st, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_rekey: NULL state");
    int rc = run_init(st, keys, ivs, iv_bits);
    if (rc != MICKEY_OK) {
        prefix_error("mickey_rekey");
        return rc;
    }
    return ok();
}

void mickey_free(mickey_state *st) { destroy(st); }

int mickey_set_stream(mickey_state *st, void *hip_stream)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_set_stream: NULL state");
    st->stream = (hipStream_t)hip_stream;
    return ok();
}

int mickey_set_word_bits(mickey_state *st, int word_bits)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_set_word_bits: NULL state");
    if (word_bits != 32 && word_bits != 64)
        return fail(MICKEY_ENOSYS, "mickey_set_word_bits: %d-bit words are not supported", word_bits);
    if (word_bits == 64 && (st->schedule == MICKEY_SCHED_SPLIT || st->schedule == MICKEY_SCHED_SPLIT4))
        return fail(MICKEY_EINVAL, "mickey_set_word_bits: the split schedule uses 32-bit words");
    st->word_bits = word_bits;
    return ok();
}

int mickey_set_transpose(mickey_state *st, int mode)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_set_transpose: NULL state");
    if (mode != MICKEY_TRANSPOSE_AUTO && mode != MICKEY_TRANSPOSE_FUSED && mode != MICKEY_TRANSPOSE_STAGED)
        return fail(MICKEY_EINVAL, "mickey_set_transpose: unknown mode %d", mode);
    st->transpose = mode;
    return ok();
}

int mickey_set_schedule(mickey_state *st, int schedule)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_set_schedule: NULL state");
    if (schedule != MICKEY_SCHED_AUTO && schedule != MICKEY_SCHED_ONE_WAVE && schedule != MICKEY_SCHED_SPLIT &&
        schedule != MICKEY_SCHED_SPLIT4)
        return fail(MICKEY_EINVAL, "mickey_set_schedule: unknown schedule %d", schedule);
    if ((schedule == MICKEY_SCHED_SPLIT || schedule == MICKEY_SCHED_SPLIT4) && st->word_bits != 32)
        return fail(MICKEY_EINVAL, "mickey_set_schedule: the split schedule uses 32-bit words");
    st->schedule = schedule;
    return ok();
}

size_t mickey_num_instances(const mickey_state *st) { return st ? st->n : 0; }

uint64_t mickey_bits_generated(const mickey_state *st) { return st ? st->bits : 0; }

uint64_t mickey_instance_bits(const mickey_state *st, size_t instance)
{
    if (!st || instance >= st->n) {
        fail(MICKEY_EINVAL, "mickey_instance_bits: NULL state or instance out of range");
        return UINT64_MAX;
    }
    ok();
    return instance_bits(st, instance);
}

size_t mickey_plane_pitch(size_t n) { return pad64(n) / 8; }

int mickey_state_export(const mickey_state *st, uint8_t *packed, uint64_t *bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "mickey_state_export: NULL argument");
    if (st->poisoned && !st->snap_valid)
        return fail(MICKEY_EDEVICE, "mickey_state_export: the state was lost to an earlier device failure");
    // a poisoned state exports the registers saved before the call that failed
    const uint32_t *regs = st->poisoned ? st->snap : st->planes;
    int rc = launch_guard("export_kernel");
    if (rc != MICKEY_OK) return rc;
    hipLaunchKernelGGL(export_kernel, dim3((unsigned)((st->n + 255) / 256)), dim3(256), 0, st->stream, regs,
                       (uint32_t)st->nslices, (uint32_t)st->n, packed);
    rc = check_launch("export_kernel");
    if (rc != MICKEY_OK) return rc;
    if (bits_generated) *bits_generated = st->bits;
    return ok();
}

int mickey_state_import(mickey_state *st, const uint8_t *packed, uint64_t bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "mickey_state_import: NULL argument");
    if (bits_generated > MICKEY_MAX_BITS_PER_IV)
        return fail(MICKEY_ERANGE, "mickey_state_import: bit counter beyond 2^40");
    int rc = launch_guard("import_kernel");
    if (rc != MICKEY_OK) return rc;
    hipLaunchKernelGGL(import_kernel, dim3((unsigned)(st->n_pad / 256 + (st->n_pad % 256 ? 1 : 0))), dim3(256), 0,
                       st->stream, packed, (uint32_t)st->n, (uint32_t)st->nslices, st->planes);
    rc = check_launch("import_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits = bits_generated;
    st->extra.clear();
    st->max_extra = 0;
    st->poisoned = false;
    st->snap_valid = false;
    return ok();
}

size_t mickey_state_host_bytes(const mickey_state *st) { return st ? host_state_bytes(st->n) : 0; }

int mickey_state_export_host(const mickey_state *st, void *host, size_t cap)
{
    if (!st || !host) return fail(MICKEY_EINVAL, "mickey_state_export_host: NULL argument");
    const size_t need = host_state_bytes(st->n);
    if (cap < need) return fail(MICKEY_EINVAL, "mickey_state_export_host: %zu bytes given, %zu needed", cap, need);
    mickey_state *w = const_cast<mickey_state *>(st);  // scratch only; the registers are read
    int rc = ensure_scratch(w, st->n * 25);
    if (rc != MICKEY_OK) return rc;
    uint8_t *packed = (uint8_t *)w->bmem;
    uint64_t bits = 0;
    rc = mickey_state_export(st, packed, &bits);
    if (rc != MICKEY_OK) return rc;
    HostHeader h;
    memcpy(h.magic, kHostMagic, 8);
    h.version = kHostVersion;
    h.state_bytes = 25;
    h.n = st->n;
    h.reserved = 0;
    char *p = (char *)host;
    memcpy(p, &h, sizeof h);
    if (hipMemcpyAsync(p + sizeof h, packed, st->n * 25, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
        hipStreamSynchronize(st->stream) != hipSuccess)
        return check_launch("mickey_state_export_host: copy to the host");
    uint8_t *cnt = (uint8_t *)p + sizeof h + st->n * 25;
    for (size_t i = 0; i < st->n; i++) {
        const uint64_t v = instance_bits(st, i);
        memcpy(cnt + 8 * i, &v, 8);
    }
    return ok();
}

int mickey_state_import_host(mickey_state *st, const void *host, size_t len)
{
    if (!st || !host) return fail(MICKEY_EINVAL, "mickey_state_import_host: NULL argument");
    const size_t need = host_state_bytes(st->n);
    HostHeader h;
    if (len < sizeof h) return fail(MICKEY_EINVAL, "mickey_state_import_host: %zu bytes is too short", len);
    memcpy(&h, host, sizeof h);
    if (memcmp(h.magic, kHostMagic, 8) != 0 || h.version != kHostVersion || h.state_bytes != 25)
        return fail(MICKEY_EINVAL, "mickey_state_import_host: not a MICKEY 2.0 state of this library");
    if (h.n != st->n)
        return fail(MICKEY_EINVAL, "mickey_state_import_host: %llu instances, the state has %zu",
                    (unsigned long long)h.n, st->n);
    if (len != need) return fail(MICKEY_EINVAL, "mickey_state_import_host: %zu bytes, expected %zu", len, need);
    const uint8_t *cnt = (const uint8_t *)host + sizeof h + st->n * 25;
    uint64_t lo = UINT64_MAX, hi = 0;
    for (size_t i = 0; i < st->n; i++) {
        uint64_t v;
        memcpy(&v, cnt + 8 * i, 8);
        if (v > MICKEY_MAX_BITS_PER_IV) return fail(MICKEY_ERANGE, "mickey_state_import_host: counter beyond 2^40");
        lo = v < lo ? v : lo;
        hi = v > hi ? v : hi;
    }
    int rc = ensure_scratch(st, st->n * 25);
    if (rc != MICKEY_OK) return rc;
    uint8_t *packed = (uint8_t *)st->bmem;
    if (hipMemcpyAsync(packed, (const uint8_t *)host + sizeof h, st->n * 25, hipMemcpyHostToDevice, st->stream) !=
            hipSuccess ||
        hipStreamSynchronize(st->stream) != hipSuccess)
        return check_launch("mickey_state_import_host: copy to the device");
    rc = mickey_state_import(st, packed, lo);
    if (rc != MICKEY_OK) return rc;
    if (hi > lo) {
        st->extra.assign(st->n, 0);
        for (size_t i = 0; i < st->n; i++) {
            uint64_t v;
            memcpy(&v, cnt + 8 * i, 8);
            st->extra[i] = v - lo;
        }
        st->max_extra = hi - lo;
    }
    return ok();
}

int mickey_sync(mickey_state *st)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_sync: NULL state");
    hipError_t e = hipStreamSynchronize(st->stream);
    if (e == hipSuccess && st->side) e = hipStreamSynchronize(st->side);
    if (e != hipSuccess) {
        st->poisoned = true;
        return fail(MICKEY_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    return ok();
}

int mickey_debug_fail_launch(int k)
{
    if (k < 0) return fail(MICKEY_EINVAL, "mickey_debug_fail_launch: k must be >= 0");
    g_fail_in.store(k);
    return ok();
}

int mickey_last_error(void) { return g_err; }

const char *mickey_last_error_message(void) { return g_msg; }

int mickey_ops_per_clock(void) { return ops_per_clock(); }

}  // extern "C"
