/*
 * aes.h - C ABI of the bitsliced AES-128 counter-mode generator in libmickey.so, on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (the paper's AES subsection of Sec. II-C: AES in counter mode, the S-box
 * evaluated as a bit-level circuit; bitsliced as in Sec. IV-D): n keystream streams under
 * one 128-bit key.  Stream i's keystream block j (j = 0, 1, ...) is
 *     AES-128_K(N_i || J),   J = j as a 64-bit big-endian integer,
 * where N_i is the stream's 8-byte nonce: the counter-block layout of NIST SP 800-38A
 * (Appendix B.2, nonce followed by a block counter, incremented in the low 64 bits).
 * 32 streams are packed one per bit lane of 32-bit words: the 128-bit AES state becomes
 * 128 words, and each round (SubBytes as the 94-operation Boyar-Peralta circuit,
 * ShiftRows as register renaming, MixColumns and AddRoundKey as XORs) runs on all lanes
 * at once.  Every output bit equals the AES standard's (FIPS-197) result.
 *
 * Conventions
 *   - The keystream of a stream is its blocks' bytes in order; keystream bit t is bit
 *     (7 - t%8) of byte t/8 (most significant first, the standards' bit order).
 *   - n is padded internally to n_pad = 64*ceil(n/64) streams (pad streams use nonce 0).
 *   - Generation advances every stream by the same number of blocks, so nbits must be a
 *     multiple of 128.
 *
 * Output layouts (aes_ctr_generate; the MICKEY_* layout codes of mickey.h):
 *   MICKEY_BITSLICED    plane t holds keystream bit t of every stream, LSB-first over
 *                       streams: stream i is bit (i % 8) of byte (t*pitch + i/8), pitch =
 *                       aes_ctr_plane_pitch(n) = n_pad/8.  Buffer: nbits*pitch bytes.
 *   MICKEY_ROWMAJOR_U32 word w of stream i is out[i*(nbits/32) + w]; bit (31 - b) of it is
 *                       keystream bit 32w + b (the word is the big-endian reading of
 *                       keystream bytes 4w..4w+3).  Buffer: n*nbits/8 bytes.
 *   MICKEY_ROWMAJOR_F32 the same words w as floats (w >> 8) * 2^-24, exact.
 *
 * Ownership, streams and errors are as for mickey_state (mickey.h): the library owns an
 * aes_ctr_state and its device memory; key and nonces are caller-owned device pointers
 * (the key is read during aes_ctr_init only); work is asynchronous on the state's stream;
 * calls on one state are not thread-safe; failures return a negative MICKEY_E* code
 * (NULL from aes_ctr_init), with mickey_last_error() / mickey_last_error_message().
 */
#ifndef AES_CTR_H
#define AES_CTR_H

#include <stddef.h>
#include <stdint.h>

#include "mickey.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aes_ctr_state aes_ctr_state;

/* Expand the 16-byte key (device) and load n 8-byte nonces (device, n*8 bytes, 8-byte
 * aligned) on hip_stream (NULL: the null stream).  Every stream starts at block 0. */
aes_ctr_state *aes_ctr_init(const uint8_t *key, const uint8_t *nonces, size_t n, void *hip_stream);

/* Advance every stream by nbits/128 blocks (nbits % 128 == 0), writing the keystream in
 * `layout` to out (device, caller-owned, sizes above).  Consecutive calls continue. */
int aes_ctr_generate(aes_ctr_state *st, uint64_t nbits, void *out, int layout);

/* Row-major delivery to u32 words, f32 values, or both (either may be NULL). */
int aes_ctr_generate_rowmajor(aes_ctr_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32);

/* Move every stream to block `block` (the next block generated).  Blocks 0 .. 2^64 - 2
 * can be generated: a call that would move the counter to 2^64 - 1 or beyond fails with
 * MICKEY_ERANGE. */
int aes_ctr_seek(aes_ctr_state *st, uint64_t block);

void aes_ctr_free(aes_ctr_state *st); /* NULL-safe; waits for the state's stream */
int aes_ctr_set_stream(aes_ctr_state *st, void *hip_stream);
size_t aes_ctr_num_instances(const aes_ctr_state *st);
uint64_t aes_ctr_bits_generated(const aes_ctr_state *st); /* 128 * next block */
size_t aes_ctr_plane_pitch(size_t n);
int aes_ctr_sync(aes_ctr_state *st);

/* VALU instructions of one block for 32 streams (algorithmic count of the circuit). */
int aes_ctr_ops_per_block(void);

#ifdef __cplusplus
}
#endif

#endif /* AES_CTR_H */
