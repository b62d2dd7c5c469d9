/*
 * Grain (version 1) reference keystream generator: plain, bit-serial, one instance at a
 * time.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU Grain path is
 * checked.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the HIP
 * library, and nothing in the product path may call it.
 *
 * What it computes.  The paper (Sec. II-C, the Grain subsection) bitslices Grain beside
 * MICKEY 2.0: an 80-bit linear register (LFSR) and an 80-bit non-linear register (NFSR)
 * shifted together once per clock, the NFSR feedback mixing in the LFSR's output, an
 * 80-bit key loaded into the NFSR and a 64-bit IV into the LFSR, and 160 initialisation
 * clocks before keystream is produced.  The paper does not restate the feedback and
 * output functions, so this file follows the cipher definition it cites (Hell, Johansson
 * and Meier's Grain specification), in that specification's notation:
 *
 *   LFSR  s_{i+80} = s_{i+62} + s_{i+51} + s_{i+38} + s_{i+23} + s_{i+13} + s_i
 *   NFSR  b_{i+80} = s_i + g(b_i .. b_{i+63})      (g written out in nfsr_feedback)
 *   output  z_i = sum_{k in A} b_{i+k} + h(s_{i+3}, s_{i+25}, s_{i+46}, s_{i+64}, b_{i+63}),
 *           A = {1, 2, 4, 10, 31, 43, 56}
 *   init    b_i = k_i (0 <= i < 80), s_i = IV_i (0 <= i < 64), s_i = 1 (64 <= i < 80);
 *           160 clocks with z_i added to both feedbacks and no output.
 *
 * Storage: reg[0] holds the oldest bit (b_i, s_i of the current clock i); a clock shifts
 * every bit down by one place and writes the new bit into reg[79].
 *
 * Bit-order conventions (those of the specification's known-answer vectors, which the
 * test suite pins): key bit k_j = bit (j%8) of key byte j/8 (least significant first),
 * the same for the IV, and keystream bit z_t goes to output byte t/8 at bit (t%8).
 *
 * Pins (in the test suite): the specification's two known-answer keystreams, primitivity
 * of the LFSR polynomial, and locality probes of the feedback and output functions.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef struct {
    uint8_t b[80]; /* NFSR b_i .. b_{i+79}, one bit per byte */
    uint8_t s[80]; /* LFSR s_i .. s_{i+79}, one bit per byte */
} gref_state;

size_t gref_state_size(void) { return sizeof(gref_state); }

/* The LFSR feedback polynomial's taps: s_{i+80} is the sum of these s_{i+k}. */
static const int LFSR_TAPS[6] = {0, 13, 23, 38, 51, 62};
/* Output taps of the NFSR that are added linearly to h. */
static const int OUT_TAPS[7] = {1, 2, 4, 10, 31, 43, 56};

int gref_lfsr_feedback(const gref_state *st)
{
    int f = 0;
    for (int k = 0; k < 6; k++) f ^= st->s[LFSR_TAPS[k]];
    return f;
}

/* g(b): the NFSR feedback without the s_i term, term by term as the specification
 * writes it. */
int gref_nfsr_g(const gref_state *st)
{
    const uint8_t *b = st->b;
    int g = b[62] ^ b[60] ^ b[52] ^ b[45] ^ b[37] ^ b[33] ^ b[28] ^ b[21] ^ b[14] ^ b[9] ^ b[0];
    g ^= b[63] & b[60];
    g ^= b[37] & b[33];
    g ^= b[15] & b[9];
    g ^= b[60] & b[52] & b[45];
    g ^= b[33] & b[28] & b[21];
    g ^= b[63] & b[45] & b[28] & b[9];
    g ^= b[60] & b[52] & b[37] & b[33];
    g ^= b[63] & b[60] & b[21] & b[15];
    g ^= b[63] & b[60] & b[52] & b[45] & b[37];
    g ^= b[33] & b[28] & b[21] & b[15] & b[9];
    g ^= b[52] & b[45] & b[37] & b[33] & b[28] & b[21];
    return g;
}

/* h(x0, x1, x2, x3, x4), the specification's filter function. */
int gref_h(int x0, int x1, int x2, int x3, int x4)
{
    return x1 ^ x4 ^ (x0 & x3) ^ (x2 & x3) ^ (x3 & x4) ^ (x0 & x1 & x2) ^ (x0 & x2 & x3) ^ (x0 & x2 & x4) ^
           (x1 & x2 & x4) ^ (x2 & x3 & x4);
}

int gref_output(const gref_state *st)
{
    int z = gref_h(st->s[3], st->s[25], st->s[46], st->s[64], st->b[63]);
    for (int k = 0; k < 7; k++) z ^= st->b[OUT_TAPS[k]];
    return z;
}

/* One clock.  In the initialisation phase (init != 0) the output bit is added to both
 * feedbacks; returns the output bit of the state before the clock. */
int gref_clock(gref_state *st, int init)
{
    const int z = gref_output(st);
    int fs = gref_lfsr_feedback(st);
    int fb = st->s[0] ^ gref_nfsr_g(st);
    if (init) {
        fs ^= z;
        fb ^= z;
    }
    memmove(st->s, st->s + 1, 79);
    memmove(st->b, st->b + 1, 79);
    st->s[79] = (uint8_t)fs;
    st->b[79] = (uint8_t)fb;
    return z;
}

/* Load key (10 bytes) and IV (8 bytes) and run the 160 initialisation clocks. */
void gref_init(gref_state *st, const uint8_t key[10], const uint8_t iv[8])
{
    for (int i = 0; i < 80; i++) st->b[i] = (key[i / 8] >> (i % 8)) & 1u;
    for (int i = 0; i < 64; i++) st->s[i] = (iv[i / 8] >> (i % 8)) & 1u;
    for (int i = 64; i < 80; i++) st->s[i] = 1;
    for (int t = 0; t < 160; t++) gref_clock(st, 1);
}

/* nbits keystream bits, packed least significant bit first into out
 * (ceil(nbits/8) bytes, zeroed here first). */
void gref_generate(gref_state *st, uint64_t nbits, uint8_t *out)
{
    memset(out, 0, (size_t)((nbits + 7) / 8));
    for (uint64_t t = 0; t < nbits; t++)
        out[t / 8] |= (uint8_t)(gref_clock(st, 0) << (t % 8));
}

/* n instances: keys n x 10 bytes, ivs n x 8 bytes; skip `skip` keystream bits, then
 * write nbits bits of instance i to out + i * ceil(nbits/8). */
void gref_generate_many(const uint8_t *keys, const uint8_t *ivs, size_t n, uint64_t skip, uint64_t nbits,
                        uint8_t *out)
{
    const size_t row = (size_t)((nbits + 7) / 8);
    for (size_t i = 0; i < n; i++) {
        gref_state st;
        gref_init(&st, keys + 10 * i, ivs + 8 * i);
        for (uint64_t t = 0; t < skip; t++) gref_clock(&st, 0);
        gref_generate(&st, nbits, out + i * row);
    }
}

/* State as 20 bytes: b_0..b_79 then s_0..s_79, bit j at byte j/8, bit (j%8). */
void gref_pack_state(const gref_state *st, uint8_t out[20])
{
    memset(out, 0, 20);
    for (int j = 0; j < 80; j++) out[j / 8] |= (uint8_t)(st->b[j] << (j % 8));
    for (int j = 0; j < 80; j++) out[10 + j / 8] |= (uint8_t)(st->s[j] << (j % 8));
}

void gref_unpack_state(gref_state *st, const uint8_t in[20])
{
    for (int j = 0; j < 80; j++) st->b[j] = (in[j / 8] >> (j % 8)) & 1u;
    for (int j = 0; j < 80; j++) st->s[j] = (in[10 + j / 8] >> (j % 8)) & 1u;
}
