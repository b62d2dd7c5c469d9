/*
 * mickey128.h - C ABI of the bitsliced MICKEY-128 2.0 generator in libmickey.so
 * (AMD Instinct MI355X, gfx950).
 *
 * The operation (paper Sec. II-C-1, which names MICKEY-128 2.0 as the 128-bit-key member
 * of the MICKEY 2.0 family, and Sec. IV-D, which bitslices independent instances one per
 * bit lane): n independent generator instances, each with its own 128-bit key and an IV
 * of 0..128 bits, packed one per bit lane of 32-bit words; the two 160-bit registers R
 * and S become 320 words per group of 32 instances, and every clock advances all lanes
 * at once.  Instance i produces exactly the keystream of the scalar construction: R with
 * the cipher's 78 feedback taps, S with the library's S tables (see below), control bits
 * c_R = s_54 ^ r_106 and c_S = s_106 ^ r_53, s_80 mixed into R's input while
 * initialising, and 160 preclocks.
 *
 * S tables.  The specification's 160-position S tables (COMP0, COMP1, FB0, FB1) were not
 * available to this library; it uses a stand-in set drawn from splitmix64 (seed 0x128)
 * with the 80-bit cipher's structure.  Keystreams therefore equal those of the published
 * MICKEY-128 2.0 only once its tables are written in; the kernels take them as
 * compile-time tables and nothing else changes.
 *
 * Conventions
 *   - Key and IV bits are read MSB first: bit j is bit (7 - j%8) of byte j/8.
 *   - z_t is keystream bit t of an instance (t = 0 is the first bit after the 160
 *     preclocks of the initialisation).
 *   - n is padded internally to n_pad = 2048*ceil(n/2048) instances (64 slices of 32, one
 *     workgroup's share); pad instances run with an all-zero key and a zero 128-bit IV.
 *
 * Output layout (mickey128_generate): plane-major bit-planes.  Plane t holds z_t of every
 * instance as an LSB-first bit vector of n_pad bits: instance i is bit (i % 8) of byte
 * (t*pitch + i/8), pitch = mickey128_plane_pitch(n) = n_pad/8 bytes.  The buffer is
 * nbits*pitch bytes; bits of pad instances are not part of the result.
 *
 * Ownership and ordering: the library owns a mickey128_state and its device memory; the
 * caller owns keys, IVs, lengths and outputs (device pointers on the current device).
 * Work runs on the state's HIP stream, asynchronously unless stated; results are valid
 * after that stream synchronises (mickey128_sync).  Calls on one state are not
 * thread-safe.
 *
 * Errors: functions return MICKEY_OK (0) or a negative MICKEY_* code from mickey.h, and
 * mickey128_init returns NULL on error; mickey_last_error() and
 * mickey_last_error_message() of the same library describe the calling thread's last
 * failure.  A generate whose launch is refused leaves the registers and bit counter
 * unchanged; a device failure reported by mickey128_sync poisons the state (every later
 * generate returns MICKEY_EDEVICE).
 */
#ifndef MICKEY128_H
#define MICKEY128_H

#include <stddef.h>
#include <stdint.h>

#include "mickey.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mickey128_state mickey128_state;

/* Load n instances and run the initialisation of each (paper Sec. IV-D's bitsliced input
 * handler; the cipher's key/IV loading and preclock procedure): registers cleared, then
 * the IV bits, the 128 key bits and 160 zero bits clocked in with mixing on.
 *   keys    device, n*16 bytes, key of instance i at keys + 16*i
 *   ivs     device, n*16 bytes, IV of instance i at ivs + 16*i (bits past its length
 *           are ignored)
 *   iv_bits device, n bytes, IV length of instance i in 0..128; NULL means 128 for all.
 *           When non-NULL the lengths are validated before any register is initialised
 *           from them, which synchronises the stream; a length over 128 gives
 *           MICKEY_EINVAL.
 *   n       1 .. 2^31
 *   hip_stream  the hipStream_t (as void*) the state's work runs on; NULL: null stream.
 * Returns NULL on error (see mickey_last_error). */
mickey128_state *mickey128_init(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n,
                                void *hip_stream);

/* Advance every instance by nbits >= 1 clocks and write the keystream bits it produced
 * (z = r_0 xor s_0 of the state before each clock; paper Sec. IV-D: one word per 32
 * instances per clock) to out as bit-planes (layout above; device, nbits*pitch bytes,
 * 4-byte aligned).  The next call continues with the following bit. */
int mickey128_generate(mickey128_state *st, uint64_t nbits, void *out);

/* Wait for the state's stream; MICKEY_EDEVICE (and the state poisoned) if it failed. */
int mickey128_sync(mickey128_state *st);

/* Copy the 320 register planes (plane j < 160 is r_j, 160 + j is s_j; n_pad/32 words
 * each, bit l of word g is instance 32g + l) to `planes` (device, 40*n_pad bytes),
 * asynchronously on the state's stream. */
int mickey128_export(const mickey128_state *st, uint32_t *planes);

/* Release the state (NULL-safe); waits for its stream first. */
void mickey128_free(mickey128_state *st);

size_t mickey128_num_instances(const mickey128_state *st);
/* Keystream bits every instance has produced so far. */
uint64_t mickey128_bits_generated(const mickey128_state *st);
/* Bytes per bit-plane for n instances: 2048*ceil(n/2048)/8. */
size_t mickey128_plane_pitch(size_t n);
/* VALU operations per clock per 32 instances in the kernels (518). */
int mickey128_ops_per_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* MICKEY128_H */
