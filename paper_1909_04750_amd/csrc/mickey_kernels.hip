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
#include "mickey_bitslice.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/mickey.h"

using namespace mickey;

namespace {

constexpr int kUnroll = 4;       // clocks per loop iteration of the generate kernels
constexpr int kInitClocks = 260; // 80 IV slots + 80 key bits + 100 preclocks
constexpr int kInputPlanes = 160;
constexpr int kMaskPlanes = 96;  // clocks 0..95 (lanes can only idle before clock 80)

// ------------------------------------------------------------------------ kernels

// 32x32 bit transpose: on return a[r] bit c equals the input a[c] bit r.
__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & 16) continue;
        const uint32_t x = a[i], y = a[i + 16];
        a[i] = (x & 0x0000FFFFu) | (y << 16);
        a[i + 16] = (x >> 16) | (y & 0xFFFF0000u);
    }
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & 8) continue;
        const uint32_t x = a[i], y = a[i + 8];
        a[i] = __builtin_amdgcn_bitop3_b32(x, y << 8, 0xFF00FF00u, (TA & ~TC) | (TB & TC));
        a[i + 8] = __builtin_amdgcn_bitop3_b32(y, x >> 8, 0x00FF00FFu, (TA & ~TC) | (TB & TC));
    }
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & 4) continue;
        const uint32_t x = a[i], y = a[i + 4];
        a[i] = __builtin_amdgcn_bitop3_b32(x, y << 4, 0xF0F0F0F0u, (TA & ~TC) | (TB & TC));
        a[i + 4] = __builtin_amdgcn_bitop3_b32(y, x >> 4, 0x0F0F0F0Fu, (TA & ~TC) | (TB & TC));
    }
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & 2) continue;
        const uint32_t x = a[i], y = a[i + 2];
        a[i] = __builtin_amdgcn_bitop3_b32(x, y << 2, 0xCCCCCCCCu, (TA & ~TC) | (TB & TC));
        a[i + 2] = __builtin_amdgcn_bitop3_b32(y, x >> 2, 0x33333333u, (TA & ~TC) | (TB & TC));
    }
#pragma unroll
    for (int i = 0; i < 32; i++) {
        if (i & 1) continue;
        const uint32_t x = a[i], y = a[i + 1];
        a[i] = __builtin_amdgcn_bitop3_b32(x, y << 1, 0xAAAAAAAAu, (TA & ~TC) | (TB & TC));
        a[i + 1] = __builtin_amdgcn_bitop3_b32(y, x >> 1, 0x55555555u, (TA & ~TC) | (TB & TC));
    }
}

// a1: input staging (the bitsliced input handler of Sec. IV-D).  Instance i with IV
// length L idles for d = 80 - L clocks and then takes its L IV bits (MSB first), so the
// key always enters at clock 80 in every lane: its input string is the 160-bit number
// (ivL << 80) | key read MSB first (ivL = the L-bit IV), and its "started" string is
// d zeros then ones.  A block of 256 instances (8 slices) writes these strings as
// 32-bit chunks to LDS; then one wave turns each (slice, chunk) into 32 bit-planes with
// an in-register 32x32 bit transpose and stores them.
template <bool MASKED>
__global__ __launch_bounds__(256) void stage_kernel(const uint8_t *__restrict__ keys,
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
    uint64_t kh = 0, ih = 0;
    uint32_t kl = 0, il = 0, L = 80;
    if (i < n) {
        const uint8_t *k = keys + 10ull * i;
        const uint8_t *v = ivs + 10ull * i;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            kh = (kh << 8) | k[b];
            ih = (ih << 8) | v[b];
        }
        kl = ((uint32_t)k[8] << 8) | k[9];
        il = ((uint32_t)v[8] << 8) | v[9];
        if (MASKED) {
            L = iv_bits[i];
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
    chunk[0][tid] = (uint32_t)(ivL >> 48);  // bits 159..128: clocks 0..31, MSB first
    chunk[1][tid] = (uint32_t)(lo >> 96);
    chunk[2][tid] = (uint32_t)(lo >> 64);
    chunk[3][tid] = (uint32_t)(lo >> 32);
    chunk[4][tid] = (uint32_t)lo;
    if (MASKED) {
        const uint32_t d = 80u - L;  // clocks before this lane starts
#pragma unroll
        for (int c = 0; c < kMaskChunks; c++) {
            const uint32_t first = 32u * c;  // "started" bit of clock first+b is (first+b >= d)
            chunk[kChunks + c][tid] = d <= first ? 0xFFFFFFFFu : (d >= first + 32u ? 0u : (0xFFFFFFFFu >> (d - first)));
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
    transpose32(a);  // a[r] bit l = chunk word of instance l, bit r = clock 32c' + 31 - r
    uint32_t *dst = c < (uint32_t)kChunks ? in_planes + (size_t)(32u * c) * nslices
                                          : mask_planes + (size_t)(32u * (c - kChunks)) * nslices;
#pragma unroll
    for (int r = 0; r < 32; r++) dst[(size_t)(31 - r) * nslices + slice] = a[r];
}

__device__ __forceinline__ uint32_t ld_plane(const uint32_t *base, size_t pitch, uint32_t t, uint32_t voff)
{
    return *(const uint32_t *)((const char *)base + (size_t)t * pitch + voff);
}

// a2: initialisation.  One lane per slice; R = S = 0 then 260 mixing clocks.  With
// MASKED, lanes whose IV is shorter than 80 bits stay at the zero state until their
// first IV bit (only needed when some IV length differs from 80).
template <bool MASKED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void init_kernel(
    const uint32_t *__restrict__ in_planes, const uint32_t *__restrict__ mask_planes,
    uint32_t *__restrict__ state, uint32_t nslices)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    const size_t pitch = (size_t)nslices * 4u;
    uint32_t voff = g * 4u;
    Regs<1> x;
#pragma unroll
    for (int j = 0; j < 100; j++) {
        x.r[j].w[0] = 0u;
        x.s[j].w[0] = 0u;
    }
    const Word<1> ones = {{0xFFFFFFFFu}};
    // IV part: clocks 0..79
    for (uint32_t t = 0; t < 80u; t += kUnroll) {
        Word<1> in[kUnroll], m[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            in[u].w[0] = ld_plane(in_planes, pitch, t + u, voff);
            m[u].w[0] = MASKED ? ld_plane(mask_planes, pitch, t + u, voff) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) clock_mix<1, MASKED>(x, in[u], m[u]);
    }
    // key part: clocks 80..159
    for (uint32_t t = 80u; t < 160u; t += kUnroll) {
        Word<1> in[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) in[u].w[0] = ld_plane(in_planes, pitch, t + u, voff);
#pragma unroll
        for (int u = 0; u < kUnroll; u++) clock_mix<1, false>(x, in[u], ones);
    }
    // preclocks: 100 clocks with input 0
    const Word<1> zero = {{0u}};
    for (uint32_t t = 160u; t < (uint32_t)kInitClocks; t += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++) clock_mix<1, false>(x, zero, ones);
    }
    asm volatile("" : "+v"(voff));
#pragma unroll
    for (int j = 0; j < 100; j++) {
        *(uint32_t *)((char *)state + (size_t)j * pitch + voff) = x.r[j].w[0];
        *(uint32_t *)((char *)state + (size_t)(100 + j) * pitch + voff) = x.s[j].w[0];
    }
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
    char *plane = (char *)out;
    uint64_t t = 0;
    for (; t + kUnroll <= nbits; t += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            st_word<K>(plane + voff, x.r[0] ^ x.s[0]);
            plane += pitch;
            clock_gen<K>(x);
        }
    }
    for (; t < nbits; t++) {
        st_word<K>(plane + voff, x.r[0] ^ x.s[0]);
        plane += pitch;
        clock_gen<K>(x);
    }
    store_state<K>(x, state, pitch, voff);
}

// a3 + a5 + a6: keystream clocks with delivery as per-instance row-major words.  Each
// 32 clocks a lane has 32 keystream words (one bit per instance); they are staged in
// LDS (8 KB per wave), transposed in registers so that word l holds 32 consecutive
// bits of instance 32g+l (first bit in the MSB), and stored as u32 and/or exact f32.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void gen_rowmajor_kernel(
    uint32_t *__restrict__ state, uint32_t nslices, uint32_t n, uint64_t nwords, uint32_t *__restrict__ out_u32,
    float *__restrict__ out_f32)
{
    __shared__ uint32_t zbuf[32][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + tid;
    if (g >= nslices) return;  // whole waves only: nslices is a multiple of 2, blocks of 64
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    Regs<1> x;
    load_state<1>(x, state, pitch, voff);
    const size_t row_bytes = (size_t)nwords * 4u;
    const uint32_t first = g * 32u;
    const uint32_t valid = n > first ? (n - first < 32u ? n - first : 32u) : 0u;
    for (uint64_t j = 0; j < nwords; j++) {
        for (int b0 = 0; b0 < 32; b0 += kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; u++) {
                // reversed row order: after the transpose, bit 31-b holds clock b
                zbuf[31 - (b0 + u)][tid] = (x.r[0] ^ x.s[0]).w[0];
                clock_gen<1>(x);
            }
        }
        uint32_t a[32];
#pragma unroll
        for (int b = 0; b < 32; b++) a[b] = zbuf[b][tid];
        transpose32(a);
        const size_t col = (size_t)j * 4u;
#pragma unroll
        for (int l = 0; l < 32; l++) {
            if ((uint32_t)l < valid) {
                const size_t off = (size_t)(first + l) * row_bytes + col;
                if (out_u32) *(uint32_t *)((char *)out_u32 + off) = a[l];
                if (out_f32) *(float *)((char *)out_f32 + off) = (float)(a[l] >> 8) * 0x1p-24f;
            }
        }
    }
    store_state<1>(x, state, pitch, voff);
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

struct mickey_state {
    size_t n;
    size_t n_pad;
    size_t nslices;
    uint32_t *planes = nullptr;       // device, 200 * nslices words
    uint32_t *stage = nullptr;        // device, input/mask planes + status word
    uint32_t *host_status = nullptr;  // pinned host word for the IV length check
    hipStream_t stream;
    uint64_t bits;
    int word_bits;
    int device;
};

namespace {

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

size_t pad64(size_t n) { return (n + 63) / 64 * 64; }

// Largest instance count the 32-bit indexing of the kernels supports.
constexpr size_t kMaxInstances = (size_t)1 << 31;

// a1 + a2 on an allocated state: stage the inputs, run the 260 initialisation clocks,
// reset the bit counter.  With iv_bits the lengths are validated (stream sync).
int run_init(mickey_state *st, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits)
{
    if (!keys || !ivs) return fail(MICKEY_EINVAL, "keys and ivs must be device pointers");
    uint32_t *in_planes = st->stage;
    uint32_t *mask_planes = st->stage + (size_t)kInputPlanes * st->nslices;
    uint32_t *status = mask_planes + (size_t)kMaskPlanes * st->nslices;
    if (hipMemsetAsync(status, 0, 4, st->stream) != hipSuccess) return check_launch("hipMemsetAsync");
    const dim3 sgrid((unsigned)((st->n_pad + 255) / 256));
    if (iv_bits)
        hipLaunchKernelGGL(stage_kernel<true>, sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits, (uint32_t)st->n,
                           (uint32_t)st->nslices, in_planes, mask_planes, status);
    else
        hipLaunchKernelGGL(stage_kernel<false>, sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits,
                           (uint32_t)st->n, (uint32_t)st->nslices, in_planes, mask_planes, status);
    int rc = check_launch("stage_kernel");
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
    if (iv_bits) {
        if (hipMemcpyAsync(st->host_status, status, 4, hipMemcpyDeviceToHost, st->stream) != hipSuccess ||
            hipStreamSynchronize(st->stream) != hipSuccess)
            return check_launch("IV length check");
        if (*st->host_status) return fail(MICKEY_EINVAL, "an IV length exceeds 80 bits");
    }
    st->bits = 0;
    return MICKEY_OK;
}

void destroy(mickey_state *st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->stream);
    if (st->planes) (void)hipFree(st->planes);
    if (st->stage) (void)hipFree(st->stage);
    if (st->host_status) (void)hipHostFree(st->host_status);
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
    hipGetDevice(&st->device);
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
    if (rc != MICKEY_OK) {
        const int code = g_err;
        char msg[sizeof g_msg];
        memcpy(msg, g_msg, sizeof msg);
        destroy(st);
        g_err = code;
        snprintf(g_msg, sizeof g_msg, "mickey_init: %s", msg);
        return nullptr;
    }
    ok();
    return st;
}

int generate_impl(mickey_state *st, uint64_t nbits, int layout, void *out, uint32_t *out_u32, float *out_f32)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_generate: NULL state");
    if (nbits == 0) return fail(MICKEY_EINVAL, "mickey_generate: nbits must be >= 1");
    if (nbits > MICKEY_MAX_BITS_PER_IV || st->bits > MICKEY_MAX_BITS_PER_IV - nbits)
        return fail(MICKEY_ERANGE, "mickey_generate: %llu + %llu bits exceeds 2^40 per key/IV pair",
                    (unsigned long long)st->bits, (unsigned long long)nbits);
    const size_t pitch = st->nslices * 4;
    if (layout == MICKEY_BITSLICED) {
        if (!out) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        if (st->word_bits == 32) {
            hipLaunchKernelGGL(gen_bitsliced_kernel<1>, dim3((unsigned)((st->nslices + 63) / 64)), dim3(64), 0,
                               st->stream, st->planes, (uint32_t)st->nslices, (uint32_t)pitch, nbits,
                               (uint32_t *)out);
        } else {
            const size_t ngroups = st->nslices / 2;
            hipLaunchKernelGGL(gen_bitsliced_kernel<2>, dim3((unsigned)((ngroups + 63) / 64)), dim3(64), 0,
                               st->stream, st->planes, (uint32_t)ngroups, (uint32_t)pitch, nbits,
                               (uint32_t *)out);
        }
        int rc = check_launch("gen_bitsliced_kernel");
        if (rc != MICKEY_OK) return rc;
    } else {
        if (nbits % 32 != 0) return fail(MICKEY_EINVAL, "row-major layouts need nbits %% 32 == 0");
        if (!out_u32 && !out_f32) return fail(MICKEY_EINVAL, "mickey_generate: NULL output");
        hipLaunchKernelGGL(gen_rowmajor_kernel, dim3((unsigned)((st->nslices + 63) / 64)), dim3(64), 0,
                           st->stream, st->planes, (uint32_t)st->nslices, (uint32_t)st->n, nbits / 32, out_u32,
                           out_f32);
        int rc = check_launch("gen_rowmajor_kernel");
        if (rc != MICKEY_OK) return rc;
    }
    st->bits += nbits;
    return ok();
}

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

int mickey_rekey(mickey_state *st, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_rekey: NULL state");
    int rc = run_init(st, keys, ivs, iv_bits);
    return rc == MICKEY_OK ? ok() : rc;
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
    st->word_bits = word_bits;
    return ok();
}

size_t mickey_num_instances(const mickey_state *st) { return st ? st->n : 0; }

uint64_t mickey_bits_generated(const mickey_state *st) { return st ? st->bits : 0; }

size_t mickey_plane_pitch(size_t n) { return pad64(n) / 8; }

int mickey_state_export(const mickey_state *st, uint8_t *packed, uint64_t *bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "mickey_state_export: NULL argument");
    hipLaunchKernelGGL(export_kernel, dim3((unsigned)((st->n + 255) / 256)), dim3(256), 0, st->stream, st->planes,
                       (uint32_t)st->nslices, (uint32_t)st->n, packed);
    int rc = check_launch("export_kernel");
    if (rc != MICKEY_OK) return rc;
    if (bits_generated) *bits_generated = st->bits;
    return ok();
}

int mickey_state_import(mickey_state *st, const uint8_t *packed, uint64_t bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "mickey_state_import: NULL argument");
    if (bits_generated > MICKEY_MAX_BITS_PER_IV)
        return fail(MICKEY_ERANGE, "mickey_state_import: bit counter beyond 2^40");
    hipLaunchKernelGGL(import_kernel, dim3((unsigned)(st->n_pad / 256 + (st->n_pad % 256 ? 1 : 0))), dim3(256), 0,
                       st->stream, packed, (uint32_t)st->n, (uint32_t)st->nslices, st->planes);
    int rc = check_launch("import_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits = bits_generated;
    return ok();
}

int mickey_sync(mickey_state *st)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_sync: NULL state");
    hipError_t e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return ok();
}

int mickey_last_error(void) { return g_err; }

const char *mickey_last_error_message(void) { return g_msg; }

int mickey_ops_per_clock(void) { return ops_per_clock(); }

}  // extern "C"
