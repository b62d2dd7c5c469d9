/*
 * MICKEY 2.0 reference keystream generator: plain, bit-serial, one instance at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the GPU path is
 * checked.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the HIP
 * library, and nothing in the product path may call it.
 *
 * What it computes.  The paper (Sec. II-C-1) uses MICKEY 2.0 by Babbage and Dodd as its
 * generator: two 100-bit registers, R (linear) and S (non-linear), each clocked
 * irregularly under control of the other; at most 2^40 keystream bits per key/IV pair.
 * Sec. IV-D packs 32 independent instances into the bit lanes of a word; that changes
 * only the data layout, so each lane must produce exactly the keystream of one scalar
 * instance.  The paper does not restate the cipher, so this file follows the cipher
 * definition it cites (the MICKEY 2.0 specification): the register update procedures
 * CLOCK_R, CLOCK_S and CLOCK_KG, the key/IV loading and preclock procedure, and the
 * keystream procedure, in that specification's order and notation.
 *
 * Bit-order conventions (the paper is silent; these are the specification's
 * known-answer conventions):
 *   - key bit k_j   = bit (7 - j%8) of key byte j/8   (MSB first), j = 0..79
 *   - IV  bit iv_j  = bit (7 - j%8) of IV  byte j/8   (MSB first), j = 0..iv_bits-1
 *   - keystream bit z_t is packed into output byte t/8 at bit (7 - t%8)  (MSB first)
 *
 * Pins (in the test suite): the specification's known-answer keystreams; primitivity
 * of the R feedback polynomial and the specification's jump property for control
 * bit 1 (x^J = x + 1 with J = 2^50 - 157); locality probes of CLOCK_S and CLOCK_KG.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef struct {
    uint8_t r[100]; /* r_0 .. r_99, one bit per byte */
    uint8_t s[100]; /* s_0 .. s_99, one bit per byte */
} mref_state;

/* R feedback tap positions (the specification's RTAPS set). */
static const int RTAPS[50] = {
     0,  1,  3,  4,  5,  6,  9, 12, 13, 16, 19, 20, 21, 22, 25, 28, 37, 38, 41, 42,
    45, 46, 50, 52, 54, 56, 58, 60, 61, 63, 64, 65, 66, 67, 71, 72, 79, 80, 81, 82,
    87, 88, 89, 90, 91, 92, 94, 95, 96, 97};

/* The specification's S-register tables, written out position by position, i = 0..99.
 * COMP0_i and COMP1_i are only defined for 1 <= i <= 98 ('-' elsewhere). */
static const char COMP0[] =
    "-0001100010111101001"   /*  0..19 */
    "01010101011010010000"   /* 20..39 */
    "00010101010000101001"   /* 40..59 */
    "11100101011111111101"   /* 60..79 */
    "0111111010100000011-";  /* 80..99 */
static const char COMP1[] =
    "-1011001011110010100"
    "01101011101111000110"
    "10111000010001011100"
    "01111110101110111100"
    "0100001110001001100-";
static const char FB0[] =
    "11110101111111100101"
    "11111111100110000001"
    "11001001010100101111"
    "01010100000000011010"
    "00110111001110011000";
static const char FB1[] =
    "11101110000111010011"
    "00010011001011000110"
    "00001101100010001001"
    "00101101010010100011"
    "11011111000000100001";

static int tab(const char *t, int i) { return t[i] == '1'; }

/* CLOCK_R(R, INPUT_BIT_R, CONTROL_BIT_R): shift up by one, feed r_99 ^ input back into
 * the tap positions, and when the control bit is set also add the pre-clock register
 * into itself (a "jump" of the linear register). */
void mref_clock_r(mref_state *st, int input_bit_r, int control_bit_r)
{
    uint8_t r_new[100];
    int feedback_bit = st->r[99] ^ (input_bit_r & 1);
    r_new[0] = 0;
    for (int i = 1; i < 100; i++)
        r_new[i] = st->r[i - 1];
    for (int k = 0; k < 50; k++)
        r_new[RTAPS[k]] ^= (uint8_t)feedback_bit;
    if (control_bit_r & 1)
        for (int i = 0; i < 100; i++)
            r_new[i] ^= st->r[i];
    memcpy(st->r, r_new, sizeof r_new);
}

/* CLOCK_S(S, INPUT_BIT_S, CONTROL_BIT_S): the non-linear intermediate s-hat, then the
 * feedback s_99 ^ input added into the positions selected by FB0 (control 0) or FB1
 * (control 1). */
void mref_clock_s(mref_state *st, int input_bit_s, int control_bit_s)
{
    uint8_t s_hat[100], s_new[100];
    int feedback_bit = st->s[99] ^ (input_bit_s & 1);
    s_hat[0] = 0;
    for (int i = 1; i <= 98; i++)
        s_hat[i] = st->s[i - 1] ^ ((st->s[i] ^ tab(COMP0, i)) & (st->s[i + 1] ^ tab(COMP1, i)));
    s_hat[99] = st->s[98];
    for (int i = 0; i < 100; i++) {
        int fb = (control_bit_s & 1) ? tab(FB1, i) : tab(FB0, i);
        s_new[i] = s_hat[i] ^ (uint8_t)(fb & feedback_bit);
    }
    memcpy(st->s, s_new, sizeof s_new);
}

/* CLOCK_KG(R, S, MIXING, INPUT_BIT): control bits from the pre-clock state, then both
 * registers clocked.  With mixing on, s_50 is added to R's input. */
void mref_clock_kg(mref_state *st, int mixing, int input_bit)
{
    int control_bit_r = st->s[34] ^ st->r[67];
    int control_bit_s = st->s[67] ^ st->r[33];
    int input_bit_r = mixing ? ((input_bit & 1) ^ st->s[50]) : (input_bit & 1);
    int input_bit_s = input_bit & 1;
    mref_clock_r(st, input_bit_r, control_bit_r);
    mref_clock_s(st, input_bit_s, control_bit_s);
}

static int get_bit_msb_first(const uint8_t *bytes, unsigned j)
{
    return (bytes[j >> 3] >> (7 - (j & 7))) & 1;
}

/* Key and IV loading, then 100 preclocks: registers start at zero; the IV bits, then
 * the 80 key bits, then 100 zero bits are fed through CLOCK_KG with mixing on.
 * Returns 0, or -1 if iv_bits > 80. */
int mref_init(mref_state *st, const uint8_t *key, const uint8_t *iv, unsigned iv_bits)
{
    if (iv_bits > 80)
        return -1;
    memset(st, 0, sizeof *st);
    for (unsigned i = 0; i < iv_bits; i++)
        mref_clock_kg(st, 1, get_bit_msb_first(iv, i));
    for (unsigned i = 0; i < 80; i++)
        mref_clock_kg(st, 1, get_bit_msb_first(key, i));
    for (unsigned i = 0; i < 100; i++)
        mref_clock_kg(st, 1, 0);
    return 0;
}

/* Keystream: each output bit is z = r_0 ^ s_0 of the current state, after which the
 * generator is clocked once with mixing off and input 0.  Writes nbits bits packed
 * MSB first into out (ceil(nbits/8) bytes; trailing bits of the last byte are 0). */
void mref_generate(mref_state *st, uint64_t nbits, uint8_t *out)
{
    memset(out, 0, (size_t)((nbits + 7) / 8));
    for (uint64_t t = 0; t < nbits; t++) {
        int z = st->r[0] ^ st->s[0];
        out[t >> 3] |= (uint8_t)(z << (7 - (t & 7)));
        mref_clock_kg(st, 0, 0);
    }
}

/* Many independent instances, one after another: instance i uses key i (10 bytes at
 * keys + 10*i) and IV i (10 bytes at ivs + 10*i, of which iv_bits[i] bits are used;
 * iv_bits == NULL means 80 for every instance), skips `skip` keystream bits, and
 * writes the next nbits bits to out + i*ceil(nbits/8).  Returns 0 or -1 (bad IV
 * length). */
int mref_generate_many(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits,
                       size_t n, uint64_t skip, uint64_t nbits, uint8_t *out)
{
    size_t row = (size_t)((nbits + 7) / 8);
    mref_state st;
    for (size_t i = 0; i < n; i++) {
        unsigned L = iv_bits ? iv_bits[i] : 80u;
        if (mref_init(&st, keys + 10 * i, ivs + 10 * i, L) != 0)
            return -1;
        for (uint64_t t = 0; t < skip; t++)
            mref_clock_kg(&st, 0, 0);
        mref_generate(&st, nbits, out + i * row);
    }
    return 0;
}

/* The 200 state bits as 25 bytes: bit j of the string r_0..r_99 s_0..s_99 goes to byte
 * j/8 at bit (7 - j%8). */
void mref_pack_state(const mref_state *st, uint8_t out[25])
{
    memset(out, 0, 25);
    for (int j = 0; j < 200; j++) {
        int b = j < 100 ? st->r[j] : st->s[j - 100];
        out[j >> 3] |= (uint8_t)(b << (7 - (j & 7)));
    }
}

void mref_unpack_state(mref_state *st, const uint8_t in[25])
{
    for (int j = 0; j < 200; j++) {
        int b = get_bit_msb_first(in, (unsigned)j);
        if (j < 100)
            st->r[j] = (uint8_t)b;
        else
            st->s[j - 100] = (uint8_t)b;
    }
}

size_t mref_state_size(void) { return sizeof(mref_state); }
