// Bitsliced AES-128 in counter mode on gfx950.  One thread owns a slice of 32 streams:
// bit l of every word belongs to stream 32*slice + l, and the AES state is 128 words
// (plane 8k + b = bit b, most significant first, of state byte k in FIPS-197 order,
// byte k = row k%4, column k/4).  A round is
//   SubBytes     16 S-box circuits (aes_sbox.h, 94 bitop3 each),
//   ShiftRows    free: each S-box writes straight into its shifted position,
//   MixColumns   per column u_r = a_r ^ a_{r+1}, out_r = xtime(u_r) ^ a_{r+1} ^ u_{r+2},
//   AddRoundKey  XOR with the round key bit, wave-uniform (scalar operand).
// The key is common to all streams, so round keys live in scalar registers.  The nonce
// half of the first counter block is fixed per stream, so its first-round S-box outputs
// are computed once per call; the counter half is common to all streams of a block, so
// its first-round S-box values are scalar table lookups.
#include "aes_sbox.h"
#include "bitmatrix.h"
#include "mickey_host.h"

#include "../../include/aes.h"

#include <hip/hip_runtime.h>

#include <new>

using namespace mickey_host;

namespace {

using aesbs::op3;
using bitops::TA;
using bitops::TB;
using bitops::TC;
using bitops::transpose32;

constexpr size_t kMaxInstances = (size_t)1 << 31;
constexpr int kXor3 = TA ^ TB ^ TC;

// ---------------------------------------------------------------------------------
// GF(2^8) modulo x^8 + x^4 + x^3 + x + 1 and the S-box byte map (FIPS-197 Sec. 5.1.1:
// multiplicative inverse, then the affine map with constant {63}), evaluated at compile
// time for the key schedule and the scalar first-round lookups.
constexpr uint8_t gf_mul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1) p ^= a;
        a = (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1B : 0));
        b >>= 1;
    }
    return p;
}

constexpr uint8_t gf_inv(uint8_t a)
{
    uint8_t r = 1, x = a;
    for (int e = 254; e; e >>= 1) {  // a^254 by square-and-multiply
        if (e & 1) r = gf_mul(r, x);
        x = gf_mul(x, x);
    }
    return a ? r : 0;
}

constexpr uint8_t rotl8(uint8_t x, int s) { return (uint8_t)((x << s) | (x >> (8 - s))); }

constexpr uint8_t sbox_byte(uint8_t a)
{
    const uint8_t b = gf_inv(a);
    return (uint8_t)(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63);
}

struct SboxTable {
    uint8_t v[256];
};

constexpr SboxTable make_sbox_table()
{
    SboxTable t{};
    for (int a = 0; a < 256; a++) t.v[a] = sbox_byte((uint8_t)a);
    return t;
}

__constant__ const SboxTable kSbox = make_sbox_table();
static_assert(make_sbox_table().v[0x53] == 0xED && make_sbox_table().v[0] == 0x63, "S-box byte map");

// Round-key bit as a word of equal bits: 0 or all ones.
__device__ __forceinline__ uint32_t key_mask(uint32_t byte, int bit)
{
    return 0u - ((byte >> (7 - bit)) & 1u);
}

// ---------------------------------------------------------------------------------
// Key expansion (FIPS-197 Sec. 5.2), one thread: 44 words into rk[176].
__global__ void aes_expand_kernel(const uint8_t *__restrict__ key, uint8_t *__restrict__ rk)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int i = 0; i < 16; i++) rk[i] = key[i];
    uint8_t rcon = 1;
    for (int i = 4; i < 44; i++) {
        uint8_t t[4] = {rk[4 * i - 4], rk[4 * i - 3], rk[4 * i - 2], rk[4 * i - 1]};
        if (i % 4 == 0) {
            const uint8_t t0 = t[0];
            t[0] = (uint8_t)(kSbox.v[t[1]] ^ rcon);
            t[1] = kSbox.v[t[2]];
            t[2] = kSbox.v[t[3]];
            t[3] = kSbox.v[t0];
            rcon = gf_mul(rcon, 2);
        }
        for (int k = 0; k < 4; k++) rk[4 * i + k] = (uint8_t)(rk[4 * i - 16 + k] ^ t[k]);
    }
}

// Nonce planes: plane p = 8k + b (k = nonce byte 0..7, b = bit, MSB first) of every slice;
// pad streams get nonce 0.
__global__ __launch_bounds__(64) void aes_nonce_kernel(const uint8_t *__restrict__ nonces, uint32_t n,
                                                       uint32_t nslices, uint32_t *__restrict__ planes)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;
    if (g >= nslices) return;
    uint32_t a[32];
#pragma unroll
    for (int w = 0; w < 2; w++) {
#pragma unroll
        for (int l = 0; l < 32; l++) {
            const uint32_t i = 32u * g + l;
            a[l] = i < n ? __builtin_bswap32(((const uint32_t *)(nonces + 8ull * i))[w]) : 0u;
        }
        transpose32(a);  // a[r] bit l = bit r of lane l's big-endian word = plane 32w + 31 - r
#pragma unroll
        for (int r = 0; r < 32; r++) planes[(size_t)(32 * w + 31 - r) * nslices + g] = a[r];
    }
}

// ---------------------------------------------------------------------------------
// Rounds.  st[k][b]: plane of bit b (MSB first) of state byte k.

// SubBytes and ShiftRows: output byte r + 4c is the S-box of input byte r + 4((c + r) % 4).
// With FINAL, the last round key (rk10, 16 bytes) is added to the outputs.
template <bool FINAL>
__device__ __forceinline__ void sub_shift(uint32_t (&st)[16][8], const uint8_t *rk10)
{
    uint32_t out[16][8];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = k % 4, c = k / 4;
        uint32_t kb[8];
#pragma unroll
        for (int b = 0; b < 8; b++) kb[b] = FINAL ? key_mask(rk10[k], b) : 0u;
        aesbs::sbox<FINAL>(st[r + 4 * ((c + r) % 4)], out[k], kb);
    }
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
        for (int b = 0; b < 8; b++) st[k][b] = out[k][b];
}

// MixColumns then AddRoundKey with round key rk (16 bytes).  Bit b of xtime(u) is
// u_{b+1}, plus u_0 where the reduction polynomial {1b} has a one (b = 3, 4, 6), and u_0
// for b = 7.
__device__ __forceinline__ void mix_add(uint32_t (&st)[16][8], const uint8_t *rk)
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        uint32_t u[4][8];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int b = 0; b < 8; b++) u[r][b] = st[4 * c + r][b] ^ st[4 * c + (r + 1) % 4][b];
        uint32_t o[4][8];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint32_t *a1 = st[4 * c + (r + 1) % 4];
            const uint32_t *u0 = u[r], *u2 = u[(r + 2) % 4];
            const uint32_t kbyte = rk[4 * c + r];
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const uint32_t km = key_mask(kbyte, b);
                if (b == 3 || b == 4 || b == 6)
                    o[r][b] = op3<kXor3>(op3<kXor3>(u0[b + 1], u0[0], a1[b]), u2[b], km);
                else
                    o[r][b] = op3<kXor3>(b == 7 ? u0[0] : u0[b + 1], a1[b], u2[b]) ^ km;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int b = 0; b < 8; b++) st[4 * c + r][b] = o[r][b];
    }
}

// First-round S-box outputs of the nonce bytes, word 8k + b (byte k, bit b) of each lane.
// They are constant for the call and read once per block, so they live in LDS (16 KiB per
// 64-lane workgroup, 128 KiB per CU at two waves per SIMD): held in registers beside a
// round's working set, they were spilled to scratch and reloaded every block.
using PreLds = uint32_t[64][64];

#define AES_ST(k, b) st[k][b]
#include "aes_rounds.inc"

// One block for the slice: counter block N_i || J under round keys rk (176 bytes);
// pre[8k + b][lane] (k < 8) are the first-round S-box outputs of the nonce bytes.
__device__ __forceinline__ void encrypt_block(uint32_t (&st)[16][8], const PreLds &pre, uint32_t lane, uint64_t J,
                                              const uint8_t *rk)
{
    // round 1: SubBytes of byte k lands at the ShiftRows position of k
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int r = k % 4, c = k / 4;
        const int src = r + 4 * ((c + r) % 4);
        if (src < 8) {
#pragma unroll
            for (int b = 0; b < 8; b++) st[k][b] = pre[8 * src + b][lane];
        } else {
            const uint32_t v = kSbox.v[(uint32_t)((J >> (8 * (15 - src))) & 0xFF) ^ rk[src]];
#pragma unroll
            for (int b = 0; b < 8; b++) st[k][b] = key_mask(v, b);
        }
    }
    mix_add(st, rk + 16);
    // rounds 2..9: the generated four-round body of aes_rounds.inc (the rounds of
    // sub_shift<false> + mix_add with registers placed for the VGPR banks), twice; it
    // loads its four round keys itself from the address it is given
    static_assert(AES_ROUNDS_COUNT == 4, "rounds 2..9 are two bodies");
#pragma unroll 1
    for (int q = 0; q < 2; q++) {
        const uint8_t *rkq = rk + 16 * (2 + AES_ROUNDS_COUNT * q);
        asm volatile(AES_ROUNDS_BODY : AES_ROUNDS_STATE(AES_ST) : [rk] "s"(rkq) : AES_ROUNDS_CLOBBERS, "memory");
    }
    sub_shift<true>(st, rk + 160);
}

// First-round S-box outputs of the nonce bytes: SubBytes(N_i ^ k0), bytes 0..7, into this
// lane's column of pre (only the lane itself reads it back).
__device__ __forceinline__ void nonce_round1(PreLds &pre, uint32_t lane, const uint32_t *planes, size_t pitch_words,
                                             uint32_t g, const uint8_t *rk)
{
#pragma unroll
    for (int k = 0; k < 8; k++) {
        uint32_t u[8], zero[8], o[8];
#pragma unroll
        for (int b = 0; b < 8; b++) {
            u[b] = planes[(size_t)(8 * k + b) * pitch_words + g] ^ key_mask(rk[k], b);
            zero[b] = 0u;
        }
        aesbs::sbox<false>(u, o, zero);
#pragma unroll
        for (int b = 0; b < 8; b++) pre[8 * k + b][lane] = o[b];
    }
}

// Keystream into bit-planes: plane 128*jb + 8k + b of block jb (relative to the call).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void aes_gen_kernel(
    const uint32_t *__restrict__ nonce_planes, const uint8_t *__restrict__ rk, uint32_t nslices, uint64_t j0,
    uint64_t nblocks, uint32_t *__restrict__ out)
{
    __shared__ PreLds pre;
    const uint32_t lane = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + lane;
    if (g >= nslices) return;
    nonce_round1(pre, lane, nonce_planes, nslices, g, rk);
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    char *plane = (char *)out;  // wave-uniform
    for (uint64_t jb = 0; jb < nblocks; jb++) {
        uint32_t st[16][8];
        encrypt_block(st, pre, lane, j0 + jb, rk);
#pragma unroll
        for (int k = 0; k < 16; k++)
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const __amdgpu_buffer_rsrc_t rs =
                    __builtin_amdgcn_make_buffer_rsrc(plane, (short)0, 0x7FFFFFFF, 0x00020000);
                __builtin_amdgcn_raw_buffer_store_b32(st[k][b], rs, (int)voff, 0, 0);
                plane += pitch;
            }
    }
}

// Keystream as per-stream row-major words: word 4*jb + q of block jb is the big-endian
// reading of its bytes 4q..4q+3, i.e. bit 31 - b of it is plane 32q + b.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void aes_rowmajor_kernel(
    const uint32_t *__restrict__ nonce_planes, const uint8_t *__restrict__ rk, uint32_t nslices, uint32_t n,
    uint64_t j0, uint64_t nblocks, uint32_t *__restrict__ out_u32, float *__restrict__ out_f32)
{
    __shared__ PreLds pre;
    const uint32_t lane = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + lane;
    if (g >= nslices) return;
    nonce_round1(pre, lane, nonce_planes, nslices, g, rk);
    const uint32_t first = 32u * g;
    const uint32_t valid = n > first ? (n - first < 32u ? n - first : 32u) : 0u;
    const size_t nwords = (size_t)nblocks * 4u;
    uint32_t *ou = out_u32 ? out_u32 + (size_t)first * nwords : nullptr;
    float *of = out_f32 ? out_f32 + (size_t)first * nwords : nullptr;
    for (uint64_t jb = 0; jb < nblocks; jb++) {
        uint32_t st[16][8];
        encrypt_block(st, pre, lane, j0 + jb, rk);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            uint32_t a[32];
#pragma unroll
            for (int b = 0; b < 32; b++) a[31 - b] = st[4 * q + b / 8][b % 8];
            transpose32(a);  // a[l] bit 31 - b = plane 32q + b of lane l
#pragma unroll
            for (int l = 0; l < 32; l++) {
                if ((uint32_t)l < valid) {
                    const size_t at = (size_t)l * nwords + 4 * jb + q;
                    if (ou) ou[at] = a[l];
                    if (of) of[at] = (float)(a[l] >> 8) * 0x1p-24f;
                }
            }
        }
    }
}

// Algorithmic VALU ops per block for 32 streams: 9 SubBytes layers of 16 S-boxes
// (the first round's are precomputed or scalar), 9 MixColumns with AddRoundKey
// (per column 32 for u and 2 per output bit), and the last round key folded into the
// S-box outputs (one extra op for each output computed from three operands: 5 per S-box).
constexpr int ops_per_block() { return 9 * 16 * aesbs::kSboxOps + 9 * 4 * (32 + 2 * 32) + 16 * 5; }

}  // namespace

struct aes_ctr_state {
    size_t n = 0, n_pad = 0, nslices = 0;
    uint32_t *nonce_planes = nullptr;  // device, 64 * nslices words
    uint8_t *rk = nullptr;             // device, 176 bytes of round keys
    hipStream_t stream = nullptr;
    uint64_t block = 0;  // next block of every stream
};

namespace {

dim3 slice_grid(const aes_ctr_state *st) { return dim3((unsigned)((st->nslices + 63) / 64)); }

void destroy(aes_ctr_state *st)
{
    if (!st) return;
    (void)hipStreamSynchronize(st->stream);
    if (st->nonce_planes) (void)hipFree(st->nonce_planes);
    if (st->rk) (void)hipFree(st->rk);
    delete st;
}

int check_blocks(const aes_ctr_state *st, uint64_t nbits)
{
    if (nbits % 128) return fail(MICKEY_EINVAL, "aes_ctr: nbits must be a multiple of 128 (whole blocks)");
    if (nbits / 128 > ~st->block) return fail(MICKEY_ERANGE, "aes_ctr: the 64-bit block counter would wrap");
    return MICKEY_OK;
}

}  // namespace

extern "C" {

aes_ctr_state *aes_ctr_init(const uint8_t *key, const uint8_t *nonces, size_t n, void *hip_stream)
{
    if (!key || !nonces) {
        fail(MICKEY_EINVAL, "aes_ctr_init: key and nonces must be device pointers");
        return nullptr;
    }
    if (n == 0 || n > kMaxInstances) {
        fail(MICKEY_EINVAL, "aes_ctr_init: n must be in 1..2^31 (got %zu)", n);
        return nullptr;
    }
    if ((uintptr_t)nonces & 7u) {
        fail(MICKEY_EINVAL, "aes_ctr_init: nonces must be 8-byte aligned");
        return nullptr;
    }
    aes_ctr_state *st = new (std::nothrow) aes_ctr_state();
    if (!st) {
        fail(MICKEY_ENOMEM, "aes_ctr_init: host allocation failed");
        return nullptr;
    }
    st->n = n;
    st->n_pad = pad64(n);
    st->nslices = st->n_pad / 32;
    st->stream = (hipStream_t)hip_stream;
    if (hipMalloc(&st->nonce_planes, 64 * st->nslices * 4) != hipSuccess || hipMalloc(&st->rk, 256) != hipSuccess) {
        (void)hipGetLastError();
        destroy(st);
        fail(MICKEY_ENOMEM, "aes_ctr_init: cannot allocate device memory");
        return nullptr;
    }
    hipLaunchKernelGGL(aes_expand_kernel, dim3(1), dim3(64), 0, st->stream, key, st->rk);
    int rc = check_launch("aes_expand_kernel");
    if (rc == MICKEY_OK) {
        hipLaunchKernelGGL(aes_nonce_kernel, slice_grid(st), dim3(64), 0, st->stream, nonces, (uint32_t)n,
                           (uint32_t)st->nslices, st->nonce_planes);
        rc = check_launch("aes_nonce_kernel");
    }
    if (rc != MICKEY_OK) {
        destroy(st);
        prefix_error("aes_ctr_init");
        return nullptr;
    }
    ok();
    return st;
}

int aes_ctr_generate_rowmajor(aes_ctr_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32)
{
    if (!st) return fail(MICKEY_EINVAL, "aes_ctr_generate_rowmajor: NULL state");
    int rc = check_blocks(st, nbits);
    if (rc != MICKEY_OK) return rc;
    if (!out_u32 && !out_f32) return fail(MICKEY_EINVAL, "aes_ctr_generate_rowmajor: NULL output");
    if (nbits == 0) return ok();
    hipLaunchKernelGGL(aes_rowmajor_kernel, slice_grid(st), dim3(64), 0, st->stream, st->nonce_planes, st->rk,
                       (uint32_t)st->nslices, (uint32_t)st->n, st->block, nbits / 128, out_u32, out_f32);
    rc = check_launch("aes_rowmajor_kernel");
    if (rc != MICKEY_OK) return rc;
    st->block += nbits / 128;
    return ok();
}

int aes_ctr_generate(aes_ctr_state *st, uint64_t nbits, void *out, int layout)
{
    if (!st) return fail(MICKEY_EINVAL, "aes_ctr_generate: NULL state");
    if (!out) return fail(MICKEY_EINVAL, "aes_ctr_generate: NULL output");
    switch (layout) {
    case MICKEY_BITSLICED: {
        int rc = check_blocks(st, nbits);
        if (rc != MICKEY_OK) return rc;
        if (nbits == 0) return ok();
        hipLaunchKernelGGL(aes_gen_kernel, slice_grid(st), dim3(64), 0, st->stream, st->nonce_planes, st->rk,
                           (uint32_t)st->nslices, st->block, nbits / 128, (uint32_t *)out);
        rc = check_launch("aes_gen_kernel");
        if (rc != MICKEY_OK) return rc;
        st->block += nbits / 128;
        return ok();
    }
    case MICKEY_ROWMAJOR_U32:
        return aes_ctr_generate_rowmajor(st, nbits, (uint32_t *)out, nullptr);
    case MICKEY_ROWMAJOR_F32:
        return aes_ctr_generate_rowmajor(st, nbits, nullptr, (float *)out);
    default:
        return fail(MICKEY_EINVAL, "aes_ctr_generate: unknown layout %d", layout);
    }
}

int aes_ctr_seek(aes_ctr_state *st, uint64_t block)
{
    if (!st) return fail(MICKEY_EINVAL, "aes_ctr_seek: NULL state");
    st->block = block;
    return ok();
}

void aes_ctr_free(aes_ctr_state *st) { destroy(st); }

int aes_ctr_set_stream(aes_ctr_state *st, void *hip_stream)
{
    if (!st) return fail(MICKEY_EINVAL, "aes_ctr_set_stream: NULL state");
    st->stream = (hipStream_t)hip_stream;
    return ok();
}

size_t aes_ctr_num_instances(const aes_ctr_state *st) { return st ? st->n : 0; }

uint64_t aes_ctr_bits_generated(const aes_ctr_state *st) { return st ? st->block * 128u : 0; }

size_t aes_ctr_plane_pitch(size_t n) { return pad64(n) / 8; }

int aes_ctr_sync(aes_ctr_state *st)
{
    if (!st) return fail(MICKEY_EINVAL, "aes_ctr_sync: NULL state");
    const hipError_t e = hipStreamSynchronize(st->stream);
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return ok();
}

int aes_ctr_ops_per_block(void) { return ops_per_block(); }

}  // extern "C"
