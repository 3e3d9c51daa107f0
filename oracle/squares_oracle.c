/*
 * CPU ORACLE for the Squares counter-based RNG (Widynski, "Squares: A Fast
 * Counter-Based RNG", arXiv 2004.06278).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * links, loads or calls it.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may use it.
 *
 * All arithmetic is on uint64_t, i.e. modulo 2^64 (C unsigned wraparound),
 * which is the arithmetic the paper's C listings are written in.  Nothing
 * here is blocked, fused, vectorised or reordered.
 *
 * Parity pins (what ties this file to the paper, not to itself) live in the
 * CPU test suite: closed forms for key 0 and for sparse power-of-two keys
 * worked by hand, the ctr = 0 reduction, the identity hi32(squares64) ==
 * squares32, the Weyl identity, counter wrap, a bit-balance screen, and a
 * mutation battery showing each plausible transcription mistake fails one
 * of them.  The counter modes are pinned against the unit-step fill
 * (subsampling, one-element fills) and special steps; the key generator by
 * hand-worked decodes, an independently written inverse and the digit
 * property.
 *
 * Parity unpinned: equality with the author's own binary and key utility,
 * which are not available.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Building blocks of one round (Section 2, Algorithm; Section 3, Discussion)
 * ------------------------------------------------------------------------ */

/* Half-square step of a round: the low 64 bits of x*x, plus a Weyl term.
 * Section 2 says only half of the square is formed; uint64_t keeps exactly
 * that half. */
static uint64_t half_square_plus(uint64_t x, uint64_t weyl)
{
    return x * x + weyl;
}

/* Circular shift by 32 bits after each square (Section 3): the random
 * middle bits move to the low half for the next round. */
static uint64_t rotate32(uint64_t x)
{
    return (x >> 32) | (x << 32);
}

/* The two Weyl terms (Section 2 and Section 3).  The Weyl sequence w += s is
 * replaced by counter * key, so the first addend is ctr*key.  The second is
 * (ctr+1)*key, which the Discussion introduces so that one of the two
 * always carries non-zero digits. */
static uint64_t weyl_y(uint64_t ctr, uint64_t key) { return ctr * key; }
static uint64_t weyl_z(uint64_t ctr, uint64_t key) { return (ctr + 1u) * key; }

/* Rounds alternate the two addends: odd rounds add y, even rounds add z
 * (both listings: rounds 1..5 add y, z, y, z, y). */
static uint64_t round_addend(int round, uint64_t y, uint64_t z)
{
    return (round % 2 == 1) ? y : z;
}

/* x entering round `last`, after rounds 1 .. last-1, each a half square plus
 * addend followed by the rotation.  x starts as y (= ctr*key). */
static uint64_t state_before_round(uint64_t y, uint64_t z, int last)
{
    uint64_t x = y;
    for (int r = 1; r < last; ++r)
        x = rotate32(half_square_plus(x, round_addend(r, y, z)));
    return x;
}

/* ------------------------------------------------------------------------
 * The two generators
 * ------------------------------------------------------------------------ */

/* squares32 (Section 2): four rounds; the output is the upper 32 bits of the
 * fourth half square.  Argument order (ctr, key) follows the paper. */
uint32_t oracle_squares32(uint64_t ctr, uint64_t key)
{
    const uint64_t y = weyl_y(ctr, key);
    const uint64_t z = weyl_z(ctr, key);
    const uint64_t x = state_before_round(y, z, 4);
    const uint64_t r4 = half_square_plus(x, round_addend(4, y, z));
    return (uint32_t)(r4 >> 32);
}

/* squares64 (Section 5): the fourth round's full 64-bit half square t is
 * kept; after rotating it, a fifth round is squared and its upper 32 bits
 * are XORed into t. */
uint64_t oracle_squares64(uint64_t ctr, uint64_t key)
{
    const uint64_t y = weyl_y(ctr, key);
    const uint64_t z = weyl_z(ctr, key);
    const uint64_t x = state_before_round(y, z, 4);
    const uint64_t t = half_square_plus(x, round_addend(4, y, z));
    const uint64_t r5 = half_square_plus(rotate32(t), round_addend(5, y, z));
    return t ^ (r5 >> 32);
}

/* Per-round trace for debugging and cross-checks: trace[r-1] is x right
 * after round r's half square (before its rotation), r = 1..5. */
void oracle_trace(uint64_t ctr, uint64_t key, uint64_t trace[5])
{
    const uint64_t y = weyl_y(ctr, key);
    const uint64_t z = weyl_z(ctr, key);
    uint64_t x = y;
    for (int r = 1; r <= 5; ++r) {
        trace[r - 1] = half_square_plus(x, round_addend(r, y, z));
        x = rotate32(trace[r - 1]);
    }
}

/* oracle_trace for m (ctr, key) pairs; trace row i is out[5i .. 5i+4]. */
void oracle_trace_batch(const uint64_t *ctrs, const uint64_t *keys, uint64_t m, uint64_t *out)
{
    for (uint64_t i = 0; i < m; ++i) oracle_trace(ctrs[i], keys[i], out + 5 * i);
}

/* ------------------------------------------------------------------------
 * Uniform conversions.  Section 5 reports floating point outputs of 53-bit
 * precision but prints no formula.  The reading used here: the top 24 bits
 * of a squares32 output scaled by 2^-24 (a float in [0,1)), and the top 53
 * bits of a squares64 output scaled by 2^-53 (a double in [0,1)).  Both are
 * exact: the integer fits the significand and the scale is a power of two.
 * ------------------------------------------------------------------------ */
float oracle_to_f32(uint32_t u)
{
    return (float)(u >> 8) * 0x1p-24f;
}

double oracle_to_f64(uint64_t u)
{
    return (double)(u >> 11) * 0x1p-53;
}

/* ------------------------------------------------------------------------
 * Bulk forms over a counter range.  Element i uses counter ctr0 + i, taken
 * modulo 2^64 (the counter is a 64-bit integer, Section 3), so a range that
 * passes 2^64 - 1 continues at 0 with the same key.
 * ------------------------------------------------------------------------ */

/* Output kinds shared with the tests (values are part of the test contract,
 * not taken from any other code).  U32X2 / F32X2 split each squares64 output
 * into two 32-bit outputs (Section 5 reports timing this split): element i
 * comes from counter ctr0 + i/2, the low half for even i and the high half for
 * odd i (the little-endian order of the 64-bit output in memory); F32X2
 * converts each half like F32. */
enum { ORACLE_U32 = 0, ORACLE_F32 = 1, ORACLE_U64 = 2, ORACLE_F64 = 3, ORACLE_U32X2 = 4, ORACLE_F32X2 = 5 };

/* The 32-bit half of squares64 that split element i uses. */
static uint32_t split_half(uint64_t key, uint64_t ctr0, uint64_t i)
{
    const uint64_t v = oracle_squares64(ctr0 + i / 2, key);
    return (i % 2 == 0) ? (uint32_t)v : (uint32_t)(v >> 32);
}

void oracle_fill_u32x2(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = split_half(key, ctr0, i);
}

void oracle_fill_f32x2(uint64_t key, uint64_t ctr0, uint64_t n, float *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_to_f32(split_half(key, ctr0, i));
}

void oracle_fill_u32(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_squares32(ctr0 + i, key);
}

void oracle_fill_u64(uint64_t key, uint64_t ctr0, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_squares64(ctr0 + i, key);
}

void oracle_fill_f32(uint64_t key, uint64_t ctr0, uint64_t n, float *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_to_f32(oracle_squares32(ctr0 + i, key));
}

void oracle_fill_f64(uint64_t key, uint64_t ctr0, uint64_t n, double *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_to_f64(oracle_squares64(ctr0 + i, key));
}

/* Width in bytes of one output of a kind, 0 for an unknown kind. */
int oracle_kind_bytes(int kind)
{
    switch (kind) {
    case ORACLE_U32: case ORACLE_F32: case ORACLE_U32X2: case ORACLE_F32X2: return 4;
    case ORACLE_U64: case ORACLE_F64: return 8;
    default: return 0;
    }
}

/* Fill `n` outputs of `kind` at `dst` (any alignment: bytes are copied). */
static int fill_kind(int kind, uint64_t key, uint64_t ctr0, uint64_t n,
                     unsigned char *dst)
{
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t c = ctr0 + i;
        switch (kind) {
        case ORACLE_U32: { uint32_t v = oracle_squares32(c, key); memcpy(dst + 4 * i, &v, 4); break; }
        case ORACLE_F32: { float v = oracle_to_f32(oracle_squares32(c, key)); memcpy(dst + 4 * i, &v, 4); break; }
        case ORACLE_U64: { uint64_t v = oracle_squares64(c, key); memcpy(dst + 8 * i, &v, 8); break; }
        case ORACLE_F64: { double v = oracle_to_f64(oracle_squares64(c, key)); memcpy(dst + 8 * i, &v, 8); break; }
        case ORACLE_U32X2: { uint32_t v = split_half(key, ctr0, i); memcpy(dst + 4 * i, &v, 4); break; }
        case ORACLE_F32X2: { float v = oracle_to_f32(split_half(key, ctr0, i)); memcpy(dst + 4 * i, &v, 4); break; }
        default: return -1;
        }
    }
    return 0;
}

/* Counter increments other than one (Section 4 tests them): element i uses
 * counter ctr0 + i*step, modulo 2^64; for the split kinds element i is word
 * i%2 of squares64 at counter ctr0 + (i/2)*step.  The second addend of each
 * round stays (ctr+1)*key: the step changes which counters are visited, not
 * the generator. */
int oracle_fill_strided(int kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                        unsigned char *out)
{
    for (uint64_t i = 0; i < n; ++i) {
        const int split = (kind == ORACLE_U32X2 || kind == ORACLE_F32X2);
        const uint64_t c = ctr0 + (split ? i / 2 : i) * step;
        switch (kind) {
        case ORACLE_U32: { uint32_t v = oracle_squares32(c, key); memcpy(out + 4 * i, &v, 4); break; }
        case ORACLE_F32: { float v = oracle_to_f32(oracle_squares32(c, key)); memcpy(out + 4 * i, &v, 4); break; }
        case ORACLE_U64: { uint64_t v = oracle_squares64(c, key); memcpy(out + 8 * i, &v, 8); break; }
        case ORACLE_F64: { double v = oracle_to_f64(oracle_squares64(c, key)); memcpy(out + 8 * i, &v, 8); break; }
        case ORACLE_U32X2: case ORACLE_F32X2: {
            const uint64_t w = oracle_squares64(c, key);
            uint32_t h = (i % 2 == 0) ? (uint32_t)w : (uint32_t)(w >> 32);
            if (kind == ORACLE_F32X2) { float f = oracle_to_f32(h); memcpy(out + 4 * i, &f, 4); }
            else memcpy(out + 4 * i, &h, 4);
            break;
        }
        default: return -1;
        }
    }
    return 0;
}

/* Key-counter mode (Section 4): the counter is fixed and the key varies;
 * output j is kind's value at counter ctr under keys[j] (kinds U32, F32,
 * U64, F64). */
int oracle_fill_keys(int kind, uint64_t ctr, const uint64_t *keys, uint64_t m, unsigned char *out)
{
    for (uint64_t j = 0; j < m; ++j) {
        switch (kind) {
        case ORACLE_U32: { uint32_t v = oracle_squares32(ctr, keys[j]); memcpy(out + 4 * j, &v, 4); break; }
        case ORACLE_F32: { float v = oracle_to_f32(oracle_squares32(ctr, keys[j])); memcpy(out + 4 * j, &v, 4); break; }
        case ORACLE_U64: { uint64_t v = oracle_squares64(ctr, keys[j]); memcpy(out + 8 * j, &v, 8); break; }
        case ORACLE_F64: { double v = oracle_to_f64(oracle_squares64(ctr, keys[j])); memcpy(out + 8 * j, &v, 8); break; }
        default: return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Distinct-digit keys (Section 3, Discussion): the upper 8 hex digits of a key
 * are mutually different, so are the lower 8, and the digits are random.
 * Reading adopted where the paper is silent: the least significant hex digit
 * is odd, so that ctr -> ctr*key is a bijection mod 2^64 (the Weyl sequence
 * behind the uniformity argument of Section 2 visits every residue only with
 * an odd increment).  The paper gives the property, not a procedure; the
 * procedure here is this library's own, with squares64 as the random source
 * so that key j is a function of (gen_key, ctr0, j) alone:
 *   the upper half of key j draws r = squares64(ctr0 + 2j, gen_key), maps it
 *   to u = floor(r * N_HI / 2^64) with N_HI = 16*15*...*9 (ordered choices of
 *   8 digits out of 16) and decodes u as the choices of a Fisher-Yates
 *   shuffle of the digits 0..15 stopped after 8 steps: step i (radix 16 - i)
 *   takes the digit at position i + (u mod radix) of the partly shuffled list
 *   and u becomes u div radix; the first digit taken is the most significant.
 *   The lower half draws r = squares64(ctr0 + 2j + 1, gen_key) and
 *   u = floor(r * N_LO / 2^64) with N_LO = 8 * 15*14*...*9; its least
 *   significant digit is the odd digit 2*(u mod 8) + 1 (u becomes u div 8),
 *   which is moved to the front of the list; steps i = 1..7 then take the
 *   other seven digits as above, most significant first.
 * ------------------------------------------------------------------------ */
#define ORACLE_KEY_CHOICES_HI 518918400ull /* 16*15*14*13*12*11*10*9 */
#define ORACLE_KEY_CHOICES_LO 259459200ull /* 8 * 15*14*13*12*11*10*9 */

/* floor(r * choices / 2^64), with the 128-bit product formed exactly. */
uint64_t oracle_key_index(uint64_t r, uint64_t choices)
{
    unsigned __int128 p = (unsigned __int128)r * choices;
    return (uint64_t)(p >> 64);
}

static void swap_digits(int *digits, int a, int b)
{
    int t = digits[a];
    digits[a] = digits[b];
    digits[b] = t;
}

/* The 8 hex digits (a 32-bit half key) that index u < N_HI selects. */
uint32_t oracle_key_upper(uint64_t u)
{
    int digits[16];
    for (int i = 0; i < 16; ++i) digits[i] = i;
    uint32_t half = 0;
    for (int i = 0; i < 8; ++i) {
        int radix = 16 - i;
        int pick = i + (int)(u % (uint64_t)radix);
        u /= (uint64_t)radix;
        swap_digits(digits, i, pick);
        half = (half << 4) | (uint32_t)digits[i];
    }
    return half;
}

/* The lower half that index u < N_LO selects: odd last digit first. */
uint32_t oracle_key_lower(uint64_t u)
{
    int digits[16];
    for (int i = 0; i < 16; ++i) digits[i] = i;
    int odd = 2 * (int)(u % 8) + 1;
    u /= 8;
    swap_digits(digits, 0, odd);
    uint32_t half = 0;
    for (int i = 1; i < 8; ++i) {
        int radix = 16 - i;
        int pick = i + (int)(u % (uint64_t)radix);
        u /= (uint64_t)radix;
        swap_digits(digits, i, pick);
        half = (half << 4) | (uint32_t)digits[i];
    }
    return (half << 4) | (uint32_t)odd;
}

int oracle_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t *keys)
{
    for (uint64_t j = 0; j < m; ++j) {
        uint64_t r_hi = oracle_squares64(ctr0 + 2 * j, gen_key);
        uint64_t r_lo = oracle_squares64(ctr0 + 2 * j + 1, gen_key);
        uint64_t upper = oracle_key_upper(oracle_key_index(r_hi, ORACLE_KEY_CHOICES_HI));
        uint64_t lower = oracle_key_lower(oracle_key_index(r_lo, ORACLE_KEY_CHOICES_LO));
        keys[j] = (upper << 32) | lower;
    }
    return 0;
}

/* Ragged batch: stream s fills lens[s] outputs of kinds[s] from counter
 * ctr0s[s] under keys[s], written at byte offset offs[s] of `out`.  This is
 * the paper's "more keys give more streams" (Section 3) laid out as one
 * output arena.  Returns 0, or -1 on an unknown kind. */
int oracle_fill_batch(uint32_t m, const uint64_t *keys, const uint64_t *ctr0s,
                      const uint64_t *lens, const uint64_t *offs,
                      const uint8_t *kinds, unsigned char *out)
{
    for (uint32_t s = 0; s < m; ++s)
        if (fill_kind(kinds[s], keys[s], ctr0s[s], lens[s], out + offs[s]) != 0)
            return -1;
    return 0;
}

/* ------------------------------------------------------------------------
 * Exact sum over a counter range (the fused consumer).  The sum is taken of
 * the integers whose scaled values are the outputs:
 *   U32: squares32          F32: squares32 >> 8   (value = sum * 2^-24)
 *   U64: squares64          F64: squares64 >> 11  (value = sum * 2^-53)
 *   U32X2: each split half  F32X2: each split half >> 8 (value = sum * 2^-24)
 * as an exact 128-bit integer, so it does not depend on summation order.
 * out[0] = low 64 bits, out[1] = high 64 bits.  Returns 0, or -1 on an
 * unknown kind.
 * ------------------------------------------------------------------------ */
int oracle_sum(int kind, uint64_t key, uint64_t ctr0, uint64_t n, uint64_t out[2])
{
    unsigned __int128 acc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t c = ctr0 + i;
        switch (kind) {
        case ORACLE_U32: acc += oracle_squares32(c, key); break;
        case ORACLE_F32: acc += oracle_squares32(c, key) >> 8; break;
        case ORACLE_U64: acc += oracle_squares64(c, key); break;
        case ORACLE_F64: acc += oracle_squares64(c, key) >> 11; break;
        case ORACLE_U32X2: acc += split_half(key, ctr0, i); break;
        case ORACLE_F32X2: acc += split_half(key, ctr0, i) >> 8; break;
        default: return -1;
        }
    }
    out[0] = (uint64_t)acc;
    out[1] = (uint64_t)(acc >> 64);
    return 0;
}
