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

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace mickey;
using namespace mickey_host;

namespace {

constexpr int kUnroll = 4;  // clocks per loop iteration of the generate kernels

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

}  // namespace mickey_host

namespace {

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
        hipLaunchKernelGGL((stage_kernel<true, false>), sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits,
                           nullptr, (uint32_t)st->n, (uint32_t)st->nslices, in_planes, mask_planes, status);
    else
        hipLaunchKernelGGL((stage_kernel<false, false>), sgrid, dim3(256), 0, st->stream, keys, ivs, iv_bits,
                           nullptr, (uint32_t)st->n, (uint32_t)st->nslices, in_planes, mask_planes, status);
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
        destroy(st);
        prefix_error("mickey_init");
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
