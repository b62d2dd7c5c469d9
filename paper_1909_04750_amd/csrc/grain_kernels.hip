// Bitsliced Grain (version 1) on gfx950: key/IV loading with the 160 initialisation
// clocks, keystream generation into bit-planes or per-instance row-major words, and
// state export/import.  One thread owns one slice of 32 instances (bit l of every word
// is instance 32*slice + l); its 160 register words stay in VGPRs for the whole call.
#include "grain_bitslice.h"
#include "mickey_host.h"

#include "../../include/grain.h"

#include <hip/hip_runtime.h>

#include <new>

using namespace grain;
using namespace mickey_host;

namespace {

constexpr size_t kMaxInstances = (size_t)1 << 31;
constexpr int kGenRings = 2;  // rings of 80 clocks per generate-loop iteration

using bitops::transpose32;

// Little-endian 32-bit word w (0..2) of the 10-byte key at p (2-byte aligned); word 2
// holds key bits 64..79 in its low half.
__device__ __forceinline__ uint32_t key_word(const uint8_t *p, int w)
{
    const uint16_t *h = (const uint16_t *)p;
    return w < 2 ? (uint32_t)h[2 * w] | ((uint32_t)h[2 * w + 1] << 16) : (uint32_t)h[4];
}

// Plane j of the state (j = 0..79: b_j, 80..159: s_j) is pitch bytes after plane j-1;
// the lane's word is at byte offset voff.
__device__ __forceinline__ void load_planes(State &x, const uint32_t *planes, size_t pitch, uint32_t voff)
{
    const char *base = (const char *)planes;
#pragma unroll
    for (int j = 0; j < kRing; j++) {
        x.b[j] = *(const uint32_t *)(base + (size_t)j * pitch + voff);
        x.s[j] = *(const uint32_t *)(base + (size_t)(kRing + j) * pitch + voff);
    }
}

// (Indexed by words: written like this the compiler keeps the clock loops free of
// spills, which it does not when the offset is laundered through an asm statement.)
// rot (wave-uniform, < 80): the window is rot clocks into a revolution, b_j and s_j in
// slot (j + rot) % 80; the planes are written in canonical order.
__device__ __forceinline__ void store_planes(const State &x, uint32_t *planes, size_t pitch_words, uint32_t g,
                                             uint32_t rot = 0)
{
#pragma unroll
    for (int k = 0; k < kRing; k++) {
        const uint32_t j = (uint32_t)k >= rot ? (uint32_t)k - rot : (uint32_t)k + kRing - rot;
        planes[(size_t)j * pitch_words + g] = x.b[k];
        planes[(size_t)(kRing + j) * pitch_words + g] = x.s[k];
    }
}

// One keystream word per clock into plane-major output through a buffer resource built
// from the wave-uniform plane address: the address arithmetic stays on the scalar unit
// and the store is a vector buffer store at the lane offset.
__device__ __forceinline__ void store_plane_word(char *plane, uint32_t voff, uint32_t z)
{
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(plane, (short)0, 0x7FFFFFFF, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b32(z, rs, (int)voff, 0, 0);
}

// Load keys and IVs of one slice into the registers (b_i = k_i, s_i = IV_i, s_64..79 = 1)
// through in-register 32x32 transposes, then run the 160 initialisation clocks (the
// paper's Grain subsection: key into the NFSR, IV into the LFSR, 160 clocks before any
// output).  Instances at or beyond n (padding) get an all-zero key and IV.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void grain_init_kernel(
    const uint8_t *__restrict__ keys, const uint8_t *__restrict__ ivs, uint32_t n, uint32_t nslices,
    uint32_t *__restrict__ planes)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    State x;
    uint32_t a[32];
#pragma unroll
    for (int w = 0; w < 3; w++) {
#pragma unroll
        for (int l = 0; l < 32; l++) {
            const uint32_t i = 32u * g + l;
            a[l] = i < n ? key_word(keys + 10ull * i, w) : 0u;
        }
        transpose32(a);  // a[r] bit l = bit r of lane l's word = key bit 32w + r
#pragma unroll
        for (int r = 0; r < 32; r++)
            if (32 * w + r < kRing) x.b[32 * w + r] = a[r];
    }
#pragma unroll
    for (int w = 0; w < 2; w++) {
#pragma unroll
        for (int l = 0; l < 32; l++) {
            const uint32_t i = 32u * g + l;
            a[l] = i < n ? ((const uint32_t *)(ivs + 8ull * i))[w] : 0u;
        }
        transpose32(a);
#pragma unroll
        for (int r = 0; r < 32; r++) x.s[32 * w + r] = a[r];
    }
#pragma unroll
    for (int r = 64; r < kRing; r++) x.s[r] = 0xFFFFFFFFu;
    auto none = [](int, uint32_t) {};
    static_assert(kInitClocks == 2 * kRing, "two rings of initialisation clocks");
    clocks80<true>(x, none);
    clocks80<true>(x, none);
    store_planes(x, planes, nslices, g);
}

// Keystream into bit-planes: plane t (pitch = nslices words) gets z_t of every instance.
#define GRAIN_LOOP_B(j) x.b[j]
#define GRAIN_LOOP_S(j) x.s[j]
#include "grain_clock_loop.inc"

// Keystream into bit-planes (RINGS is kept for the launch; the generated loop runs one ring
// revolution per iteration).
template <int RINGS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void grain_gen_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint64_t nbits, uint32_t *__restrict__ out)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    State x;
    load_planes(x, planes, pitch, voff);
    char *plane = (char *)out;  // wave-uniform
    auto emit = [&](int, uint32_t z) {
        store_plane_word(plane, voff, z);
        plane += pitch;
    };
    // One ring revolution (80 clocks) per iteration of the loop generated by
    // gen_grain_loop.py, with the ring slots in VGPRs chosen for the register banks; the
    // plane stores go through a buffer resource in s[20:23] whose base advances by the
    // pitch every clock, and s24 counts iterations.  The window is back in canonical order
    // after each revolution.
    for (uint64_t left = nbits / kRing; left != 0;) {
        const uint32_t iters = left > (1u << 30) ? (1u << 30) : (uint32_t)left;
        const uint64_t base = (uint64_t)(uintptr_t)plane;
        asm volatile("s_mov_b32 s20, %[lo]\n\t"
                     "s_and_b32 s21, %[hi], 0xffff\n\t"
                     "s_mov_b32 s22, 0x7fffffff\n\t"
                     "s_mov_b32 s23, 0x20000\n\t"
                     "s_mov_b32 s24, %[it]\n"
                     "1:\n\t" GRAIN_LOOP_BODY
                     "\ts_sub_u32 s24, s24, 1\n\t"
                     "s_cmp_lg_u32 s24, 0\n\t"
                     "s_cbranch_scc1 1b"
                     : GRAIN_LOOP_STATE(GRAIN_LOOP_B, GRAIN_LOOP_S)
                     : [lo] "s"((uint32_t)base), [hi] "s"((uint32_t)(base >> 32)), [pitch] "s"((uint32_t)pitch),
                       [it] "s"(iters), [voff] "v"(voff)
                     : GRAIN_LOOP_CLOBBERS, "s20", "s21", "s22", "s23", "s24", "scc");
        left -= iters;
        plane += (uint64_t)iters * kRing * pitch;
    }
    // the last nbits % 80 clocks: a revolution's first clocks, then the planes stored
    // back in canonical order from the rotated window
    const uint32_t rem = (uint32_t)(nbits % kRing);
    ring_prefix(x, rem, emit, std::make_integer_sequence<int, kRing>{});
    store_planes(x, planes, nslices, g, rem);
}

// 32 clocks of row-major words: zz[b] holds z of clock b for the slice (bit l = lane l);
// a 32x32 transpose gives each instance l the word whose bit b is its keystream bit
// 32j + b (least significant first, so the word's little-endian bytes are the cipher's
// byte stream).
struct RowOut {
    uint32_t *u32;
    float *f32;
    size_t nwords;
    uint32_t valid;
};

__device__ __forceinline__ void flush_words(uint32_t (&zz)[32], const RowOut &o, uint64_t j)
{
    transpose32(zz);
#pragma unroll
    for (int l = 0; l < 32; l++) {
        if ((uint32_t)l < o.valid) {
            if (o.u32) o.u32[(size_t)l * o.nwords + j] = zz[l];
            if (o.f32) o.f32[(size_t)l * o.nwords + j] = (float)(zz[l] >> 8) * 0x1p-24f;
        }
    }
}

// 160 clocks (two rings, five words) fully unrolled, so that ring slots and word
// positions are both compile-time.
template <int... C>
__device__ __forceinline__ void rows160(State &x, uint32_t (&zz)[32], const RowOut &o, uint64_t j0,
                                        std::integer_sequence<int, C...>)
{
    (([&] {
         constexpr int c = C;
         zz[c % 32] = clock_ring<c % kRing, false>(x);
         if constexpr (c % 32 == 31) flush_words(zz, o, j0 + c / 32);
     }()),
     ...);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void grain_rowmajor_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint32_t n, uint64_t nwords, uint32_t *__restrict__ out_u32,
    float *__restrict__ out_f32)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    State x;
    load_planes(x, planes, (size_t)nslices * 4u, g * 4u);
    const uint32_t first = 32u * g;
    RowOut o;
    o.valid = n > first ? (n - first < 32u ? n - first : 32u) : 0u;
    o.nwords = nwords;
    o.u32 = out_u32 ? out_u32 + (size_t)first * nwords : nullptr;
    o.f32 = out_f32 ? out_f32 + (size_t)first * nwords : nullptr;
    uint32_t zz[32];
    uint64_t j = 0;
    for (; j + 5 <= nwords; j += 5) rows160(x, zz, o, j, std::make_integer_sequence<int, 2 * kRing>{});
#pragma unroll 1
    for (; j < nwords; j++) {
#pragma unroll 1
        for (int b = 0; b < 32; b++) {
            const uint32_t z = clock_shift(x);
#pragma unroll
            for (int k = 0; k < 32; k++)
                if (k == b) zz[k] = z;  // keep zz in registers: no dynamic indexing
        }
        flush_words(zz, o, j);
    }
    store_planes(x, planes, nslices, g);
}

// State export: 20 bytes per instance, bit j of b_0..b_79 s_0..s_79 at byte j/8, bit j%8;
// one thread per slice transposes the 160 plane words into five 32-bit row words per lane.
__global__ __launch_bounds__(64) void grain_export_kernel(const uint32_t *__restrict__ planes, uint32_t nslices,
                                                           uint32_t n, uint8_t *__restrict__ packed)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    uint32_t a[32];
#pragma unroll
    for (int w = 0; w < 5; w++) {
#pragma unroll
        for (int r = 0; r < 32; r++) a[r] = planes[(size_t)(32 * w + r) * nslices + g];
        transpose32(a);  // a[l] bit r = plane 32w + r, lane l
#pragma unroll
        for (int l = 0; l < 32; l++) {
            const uint32_t i = 32u * g + l;
            if (i < n) {
                uint8_t *p = packed + 20ull * i + 4 * w;
                p[0] = (uint8_t)a[l];
                p[1] = (uint8_t)(a[l] >> 8);
                p[2] = (uint8_t)(a[l] >> 16);
                p[3] = (uint8_t)(a[l] >> 24);
            }
        }
    }
}

// State import (inverse of export); pad instances get the all-zero state.
__global__ __launch_bounds__(64) void grain_import_kernel(const uint8_t *__restrict__ packed, uint32_t n,
                                                           uint32_t nslices, uint32_t *__restrict__ planes)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    uint32_t a[32];
#pragma unroll
    for (int w = 0; w < 5; w++) {
#pragma unroll
        for (int l = 0; l < 32; l++) {
            const uint32_t i = 32u * g + l;
            uint32_t v = 0;
            if (i < n) {
                const uint8_t *p = packed + 20ull * i + 4 * w;
                v = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
            }
            a[l] = v;
        }
        transpose32(a);
#pragma unroll
        for (int r = 0; r < 32; r++) planes[(size_t)(32 * w + r) * nslices + g] = a[r];
    }
}

}  // namespace

struct grain_state {
    size_t n = 0, n_pad = 0, nslices = 0;
    uint32_t *planes = nullptr;  // device, 160 * nslices words
    hipStream_t stream = nullptr;
    uint64_t bits = 0;
};

namespace {

dim3 slice_grid(const grain_state *st) { return dim3((unsigned)((st->nslices + 63) / 64)); }

int run_init(grain_state *st, const uint8_t *keys, const uint8_t *ivs)
{
    if (!keys || !ivs) return fail(MICKEY_EINVAL, "keys and ivs must be device pointers");
    if (((uintptr_t)keys & 1u) || ((uintptr_t)ivs & 7u))
        return fail(MICKEY_EINVAL, "keys must be 2-byte and ivs 8-byte aligned");
    hipLaunchKernelGGL(grain_init_kernel, slice_grid(st), dim3(64), 0, st->stream, keys, ivs, (uint32_t)st->n,
                       (uint32_t)st->nslices, st->planes);
    int rc = check_launch("grain_init_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits = 0;
    return MICKEY_OK;
}

void destroy(grain_state *st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->stream);
    if (st->planes) (void)hipFree(st->planes);
    delete st;
}

}  // namespace

extern "C" {

grain_state *grain_init(const uint8_t *keys, const uint8_t *ivs, size_t n, void *hip_stream)
{
    if (!keys || !ivs) {
        fail(MICKEY_EINVAL, "grain_init: keys and ivs must be device pointers");
        return nullptr;
    }
    if (n == 0 || n > kMaxInstances) {
        fail(MICKEY_EINVAL, "grain_init: n must be in 1..2^31 (got %zu)", n);
        return nullptr;
    }
    grain_state *st = new (std::nothrow) grain_state();
    if (!st) {
        fail(MICKEY_ENOMEM, "grain_init: host allocation failed");
        return nullptr;
    }
    st->n = n;
    st->n_pad = pad64(n);
    st->nslices = st->n_pad / 32;
    st->stream = (hipStream_t)hip_stream;
    const size_t bytes = (size_t)2 * kRing * st->nslices * 4;
    if (hipMalloc(&st->planes, bytes) != hipSuccess) {
        (void)hipGetLastError();
        destroy(st);
        fail(MICKEY_ENOMEM, "grain_init: cannot allocate %zu bytes of device memory", bytes);
        return nullptr;
    }
    const int rc = run_init(st, keys, ivs);
    if (rc != MICKEY_OK) {
        destroy(st);
        prefix_error("grain_init");
        return nullptr;
    }
    ok();
    return st;
}

int grain_rekey(grain_state *st, const uint8_t *keys, const uint8_t *ivs)
{
    if (!st) return fail(MICKEY_EINVAL, "grain_rekey: NULL state");
    const int rc = run_init(st, keys, ivs);
    return rc == MICKEY_OK ? ok() : rc;
}

int grain_generate_rowmajor(grain_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32)
{
    if (!st) return fail(MICKEY_EINVAL, "grain_generate_rowmajor: NULL state");
    if (nbits == 0) return ok();
    if (nbits % 32) return fail(MICKEY_EINVAL, "row-major layouts need nbits %% 32 == 0");
    if (!out_u32 && !out_f32) return fail(MICKEY_EINVAL, "grain_generate_rowmajor: NULL output");
    hipLaunchKernelGGL(grain_rowmajor_kernel, slice_grid(st), dim3(64), 0, st->stream, st->planes,
                       (uint32_t)st->nslices, (uint32_t)st->n, nbits / 32, out_u32, out_f32);
    const int rc = check_launch("grain_rowmajor_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits += nbits;
    return ok();
}

int grain_generate(grain_state *st, uint64_t nbits, void *out, int layout)
{
    if (!st) return fail(MICKEY_EINVAL, "grain_generate: NULL state");
    if (!out) return fail(MICKEY_EINVAL, "grain_generate: NULL output");
    switch (layout) {
    case MICKEY_BITSLICED: {
        if (nbits == 0) return ok();
        hipLaunchKernelGGL(grain_gen_kernel<kGenRings>, slice_grid(st), dim3(64), 0, st->stream, st->planes,
                           (uint32_t)st->nslices, nbits, (uint32_t *)out);
        const int rc = check_launch("grain_gen_kernel");
        if (rc != MICKEY_OK) return rc;
        st->bits += nbits;
        return ok();
    }
    case MICKEY_ROWMAJOR_U32:
        return grain_generate_rowmajor(st, nbits, (uint32_t *)out, nullptr);
    case MICKEY_ROWMAJOR_F32:
        return grain_generate_rowmajor(st, nbits, nullptr, (float *)out);
    default:
        return fail(MICKEY_EINVAL, "grain_generate: unknown layout %d", layout);
    }
}

void grain_free(grain_state *st) { destroy(st); }

int grain_set_stream(grain_state *st, void *hip_stream)
{
    if (!st) return fail(MICKEY_EINVAL, "grain_set_stream: NULL state");
    st->stream = (hipStream_t)hip_stream;
    return ok();
}

size_t grain_num_instances(const grain_state *st) { return st ? st->n : 0; }

uint64_t grain_bits_generated(const grain_state *st) { return st ? st->bits : 0; }

size_t grain_plane_pitch(size_t n) { return pad64(n) / 8; }

int grain_state_export(const grain_state *st, uint8_t *packed, uint64_t *bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "grain_state_export: NULL argument");
    hipLaunchKernelGGL(grain_export_kernel, slice_grid(st), dim3(64), 0, st->stream, st->planes,
                       (uint32_t)st->nslices, (uint32_t)st->n, packed);
    const int rc = check_launch("grain_export_kernel");
    if (rc != MICKEY_OK) return rc;
    if (bits_generated) *bits_generated = st->bits;
    return ok();
}

int grain_state_import(grain_state *st, const uint8_t *packed, uint64_t bits_generated)
{
    if (!st || !packed) return fail(MICKEY_EINVAL, "grain_state_import: NULL argument");
    hipLaunchKernelGGL(grain_import_kernel, slice_grid(st), dim3(64), 0, st->stream, packed, (uint32_t)st->n,
                       (uint32_t)st->nslices, st->planes);
    const int rc = check_launch("grain_import_kernel");
    if (rc != MICKEY_OK) return rc;
    st->bits = bits_generated;
    return ok();
}

int grain_sync(grain_state *st)
{
    if (!st) return fail(MICKEY_EINVAL, "grain_sync: NULL state");
    const hipError_t e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return ok();
}

int grain_ops_per_clock(void) { return ops_per_clock(); }

}  // extern "C"
