/*
 * AES-128 and CTR-mode keystream reference: plain, byte-oriented, one block at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU AES-CTR path
 * is checked.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the HIP
 * library, and nothing in the product path may call it.
 *
 * What it computes.  The paper (Sec. II-C, the AES subsection) uses AES in counter mode
 * as its third generator: the 16-byte state is transformed by SubBytes (the only
 * non-linear step, which the paper evaluates as a bit-level circuit), ShiftRows,
 * MixColumns (multiplication in GF(2^8)) and AddRoundKey, 10 rounds for a 128-bit key.
 * The paper does not restate the cipher, so this file follows the AES standard (FIPS-197)
 * and the counter mode of NIST SP 800-38A:
 *   - the S-box value of a byte is the multiplicative inverse in GF(2^8) modulo
 *     x^8 + x^4 + x^3 + x + 1 (0 maps to 0), followed by the affine transform with the
 *     constant 0x63; it is computed here from that definition, not from a stored table;
 *   - the key schedule expands 4 key words to 44 with RotWord, SubWord and the round
 *     constants x^(i-1) in GF(2^8);
 *   - CTR: keystream block j of a stream is AES_K(T_j), where T_j is the initial counter
 *     block plus j as a 128-bit big-endian integer (mod 2^128).
 *
 * Pins (in the test suite): FIPS-197's example vectors, the SP 800-38A CTR-AES128
 * vectors, and algebraic properties of the S-box and of MixColumns.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* Multiplication in GF(2^8) modulo x^8 + x^4 + x^3 + x + 1, bit by bit. */
uint8_t aref_gmul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1) p ^= a;
        const int hi = a & 0x80;
        a = (uint8_t)(a << 1);
        if (hi) a ^= 0x1B;
        b >>= 1;
    }
    return p;
}

/* Multiplicative inverse: a^254 (a^(2^8 - 2)); 0 maps to 0. */
uint8_t aref_ginv(uint8_t a)
{
    uint8_t r = 1;
    for (int i = 0; i < 254; i++) r = aref_gmul(r, a);
    return a ? r : 0;
}

/* SubBytes of one byte: inverse, then b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i
 * (indices mod 8, c = 0x63). */
uint8_t aref_sbox(uint8_t a)
{
    const uint8_t b = aref_ginv(a);
    uint8_t s = 0;
    for (int i = 0; i < 8; i++) {
        const int bit = ((b >> i) ^ (b >> ((i + 4) % 8)) ^ (b >> ((i + 5) % 8)) ^ (b >> ((i + 6) % 8)) ^
                         (b >> ((i + 7) % 8)) ^ (0x63 >> i)) & 1;
        s |= (uint8_t)(bit << i);
    }
    return s;
}

/* Key expansion: 44 words of 4 bytes (w[i][0] is the most significant byte). */
void aref_expand_key(const uint8_t key[16], uint8_t w[44][4])
{
    for (int i = 0; i < 4; i++) memcpy(w[i], key + 4 * i, 4);
    uint8_t rcon = 1;
    for (int i = 4; i < 44; i++) {
        uint8_t t[4];
        memcpy(t, w[i - 1], 4);
        if (i % 4 == 0) {
            const uint8_t r0 = t[0];  /* RotWord */
            t[0] = t[1];
            t[1] = t[2];
            t[2] = t[3];
            t[3] = r0;
            for (int k = 0; k < 4; k++) t[k] = aref_sbox(t[k]);  /* SubWord */
            t[0] ^= rcon;
            rcon = aref_gmul(rcon, 2);
        }
        for (int k = 0; k < 4; k++) w[i][k] = w[i - 4][k] ^ t[k];
    }
}

/* The state as FIPS-197 lays it out: s[r][c] = in[r + 4c]. */
static void add_round_key(uint8_t s[4][4], const uint8_t w[44][4], int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++) s[r][c] ^= w[4 * round + c][r];
}

static void sub_bytes(uint8_t s[4][4])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) s[r][c] = aref_sbox(s[r][c]);
}

/* Row r is rotated left by r positions. */
static void shift_rows(uint8_t s[4][4])
{
    for (int r = 1; r < 4; r++) {
        uint8_t t[4];
        for (int c = 0; c < 4; c++) t[c] = s[r][(c + r) % 4];
        memcpy(s[r], t, 4);
    }
}

/* Each column times the polynomial {03}x^3 + {01}x^2 + {01}x + {02} modulo x^4 + 1. */
static void mix_columns(uint8_t s[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a[4];
        for (int r = 0; r < 4; r++) a[r] = s[r][c];
        for (int r = 0; r < 4; r++)
            s[r][c] = aref_gmul(a[r], 2) ^ aref_gmul(a[(r + 1) % 4], 3) ^ a[(r + 2) % 4] ^ a[(r + 3) % 4];
    }
}

void aref_encrypt_block(const uint8_t w[44][4], const uint8_t in[16], uint8_t out[16])
{
    uint8_t s[4][4];
    for (int i = 0; i < 16; i++) s[i % 4][i / 4] = in[i];
    add_round_key(s, w, 0);
    for (int round = 1; round < 10; round++) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s);
    shift_rows(s);
    add_round_key(s, w, 10);
    for (int i = 0; i < 16; i++) out[i] = s[i % 4][i / 4];
}

void aref_encrypt(const uint8_t key[16], const uint8_t in[16], uint8_t out[16])
{
    uint8_t w[44][4];
    aref_expand_key(key, w);
    aref_encrypt_block(w, in, out);
}

/* Counter block T + j, as 128-bit big-endian integers, modulo 2^128. */
void aref_counter_add(const uint8_t t[16], uint64_t j, uint8_t out[16])
{
    unsigned carry = 0;
    for (int i = 15; i >= 0; i--) {
        const unsigned add = (i >= 8) ? (unsigned)((j >> (8 * (15 - i))) & 0xFF) : 0u;
        const unsigned v = t[i] + add + carry;
        out[i] = (uint8_t)v;
        carry = v >> 8;
    }
}

/* CTR keystream of n streams under one key: stream i starts at counter block ctr0[i]
 * (16 bytes each) advanced by `skip` blocks, and gets nblocks blocks written to
 * out + 16 * nblocks * i. */
void aref_ctr_many(const uint8_t key[16], const uint8_t *ctr0, size_t n, uint64_t skip, uint64_t nblocks,
                   uint8_t *out)
{
    uint8_t w[44][4];
    aref_expand_key(key, w);
    for (size_t i = 0; i < n; i++) {
        for (uint64_t j = 0; j < nblocks; j++) {
            uint8_t t[16];
            aref_counter_add(ctr0 + 16 * i, skip + j, t);
            aref_encrypt_block(w, t, out + 16 * (nblocks * i + j));
        }
    }
}
