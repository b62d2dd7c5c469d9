/*
 * grain.h - C ABI of the bitsliced Grain (version 1) generator in libmickey.so, on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (the paper's Grain subsection of Sec. II-C, bitsliced as in Sec. IV-D):
 * n independent Grain instances, each with its own 80-bit key and 64-bit IV, are packed
 * one per bit lane of 32-bit words.  The 80-bit NFSR and 80-bit LFSR become 160 words
 * per group of 32 instances, the 160 initialisation clocks run with the output fed back
 * into both registers, and every keystream clock advances all lanes at once.  Instance i
 * produces exactly the keystream of the Grain definition the paper cites, bit for bit.
 *
 * Conventions (those of the Grain specification's known-answer vectors)
 *   - Key bit k_j is bit (j % 8) of key byte j/8 (least significant first); IV bit IV_j
 *     likewise.  Keys are 10 bytes, IVs 8 bytes, per instance, contiguous.
 *   - z_t is keystream bit t of an instance (t = 0 is the first bit after the 160
 *     initialisation clocks).
 *   - n is padded internally to n_pad = 64*ceil(n/64); pad instances run with an all-zero
 *     key and IV.
 *
 * Output layouts (grain_generate; the MICKEY_* layout codes of mickey.h):
 *   MICKEY_BITSLICED    plane t (t = 0..nbits-1) holds z_t of every instance as an
 *                       LSB-first bit vector of n_pad bits: instance i is bit (i % 8) of
 *                       byte (t*pitch + i/8), pitch = grain_plane_pitch(n) = n_pad/8
 *                       bytes.  Buffer: nbits*pitch bytes.  Pad-instance bits are not
 *                       part of the result.
 *   MICKEY_ROWMAJOR_U32 word j of instance i is out[i*(nbits/32) + j] and bit b of it is
 *                       z_{32j+b}: on a little-endian host the bytes of instance i's
 *                       words are the cipher's byte stream (bit t%8 of byte t/8 is z_t).
 *                       Needs nbits % 32 == 0.  Buffer: n*nbits/8 bytes.
 *   MICKEY_ROWMAJOR_F32 the same words w as floats (w >> 8) * 2^-24 (exact, in
 *                       [0, 1 - 2^-24]).  Needs nbits % 32 == 0.
 *
 * Ownership, streams and errors are as for mickey_state (mickey.h): the library owns a
 * grain_state and its device memory, the caller owns keys, IVs and outputs (HIP device
 * pointers; keys 2-byte aligned, IVs 8-byte aligned), work is asynchronous on the
 * state's stream, calls on one state are not thread-safe, and failures return a negative
 * MICKEY_E* code (NULL from grain_init) with mickey_last_error() /
 * mickey_last_error_message() describing it.  A failed call leaves the state unchanged.
 */
#ifndef GRAIN_H
#define GRAIN_H

#include <stddef.h>
#include <stdint.h>

#include "mickey.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct grain_state grain_state;

/* Load n keys (n*10 bytes) and IVs (n*8 bytes) and run the 160 initialisation clocks on
 * hip_stream (NULL: the null stream).  The inputs may be reused once that stream has
 * passed this call.  Returns NULL on error. */
grain_state *grain_init(const uint8_t *keys, const uint8_t *ivs, size_t n, void *hip_stream);

/* Re-initialise every instance from new keys and IVs (same n); resets the bit counter. */
int grain_rekey(grain_state *st, const uint8_t *keys, const uint8_t *ivs);

/* Advance every instance by nbits clocks, writing the keystream in `layout` to out
 * (device, caller-owned, sizes above).  Consecutive calls continue each stream. */
int grain_generate(grain_state *st, uint64_t nbits, void *out, int layout);

/* Row-major delivery to u32 words, f32 values, or both at once (either may be NULL). */
int grain_generate_rowmajor(grain_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32);

void grain_free(grain_state *st); /* NULL-safe; waits for the state's stream */

int grain_set_stream(grain_state *st, void *hip_stream);
size_t grain_num_instances(const grain_state *st);
uint64_t grain_bits_generated(const grain_state *st);
size_t grain_plane_pitch(size_t n);

/* Registers of every instance as 20 bytes (b_0..b_79 then s_0..s_79, bit j at byte j/8,
 * bit j%8; b_0 and s_0 are the bits the next clock reads first) to/from device memory
 * packed[n*20], stream-ordered; import also sets the bit counter. */
int grain_state_export(const grain_state *st, uint8_t *packed, uint64_t *bits_generated);
int grain_state_import(grain_state *st, const uint8_t *packed, uint64_t bits_generated);

int grain_sync(grain_state *st);

/* VALU instructions of one keystream clock for 32 instances. */
int grain_ops_per_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAIN_H */
