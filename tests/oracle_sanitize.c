/*
 * Test program (built with the host's address and undefined-behaviour
 * sanitizers by tests/test_oracle_pins.py): calls every entry point of the
 * CPU oracle on edge cases with output buffers of exactly the size each call
 * may write, so an out-of-range write, an overflow of a signed or shifted
 * quantity, or a read of uninitialised memory stops the run.  It also checks
 * identities that tie the entry points to each other (bulk forms against the
 * scalar functions, strided fills with step 1 against the plain fill, the
 * batch against per-stream fills, sums against element-wise sums).  Prints
 * "ok" and exits 0 when every check holds.  Host code only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint32_t oracle_squares32(uint64_t ctr, uint64_t key);
uint64_t oracle_squares64(uint64_t ctr, uint64_t key);
void oracle_trace(uint64_t ctr, uint64_t key, uint64_t trace[5]);
void oracle_trace_batch(const uint64_t *ctrs, const uint64_t *keys, uint64_t m, uint64_t *out);
float oracle_to_f32(uint32_t u);
double oracle_to_f64(uint64_t u);
int oracle_kind_bytes(int kind);
void oracle_fill_u32(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out);
void oracle_fill_f32(uint64_t key, uint64_t ctr0, uint64_t n, float *out);
void oracle_fill_u64(uint64_t key, uint64_t ctr0, uint64_t n, uint64_t *out);
void oracle_fill_f64(uint64_t key, uint64_t ctr0, uint64_t n, double *out);
void oracle_fill_u32x2(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out);
void oracle_fill_f32x2(uint64_t key, uint64_t ctr0, uint64_t n, float *out);
int oracle_fill_strided(int kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n, unsigned char *out);
int oracle_fill_keys(int kind, uint64_t ctr, const uint64_t *keys, uint64_t m, unsigned char *out);
uint64_t oracle_key_index(uint64_t r, uint64_t choices);
uint32_t oracle_key_upper(uint64_t u);
uint32_t oracle_key_lower(uint64_t u);
int oracle_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t *keys);
int oracle_fill_batch(uint32_t m, const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                      const uint64_t *offs, const uint8_t *kinds, unsigned char *out);
int oracle_sum(int kind, uint64_t key, uint64_t ctr0, uint64_t n, uint64_t out[2]);

static int failures = 0;
#define CHECK(c, ...)                     \
    do {                                  \
        if (!(c)) {                       \
            ++failures;                   \
            printf("FAIL %s: ", #c);      \
            printf(__VA_ARGS__);          \
            printf("\n");                 \
        }                                 \
    } while (0)

/* The per-kind bulk fill of the oracle; -1 for an unknown kind. */
static int oracle_fill(int kind, uint64_t key, uint64_t ctr0, uint64_t n, unsigned char *out)
{
    switch (kind) {
    case 0: oracle_fill_u32(key, ctr0, n, (uint32_t *)out); return 0;
    case 1: oracle_fill_f32(key, ctr0, n, (float *)out); return 0;
    case 2: oracle_fill_u64(key, ctr0, n, (uint64_t *)out); return 0;
    case 3: oracle_fill_f64(key, ctr0, n, (double *)out); return 0;
    case 4: oracle_fill_u32x2(key, ctr0, n, (uint32_t *)out); return 0;
    case 5: oracle_fill_f32x2(key, ctr0, n, (float *)out); return 0;
    default: return -1;
    }
}

/* Exactly n bytes (at least one, so that malloc(0) is never asked for). */
static unsigned char *exact(uint64_t n) { return (unsigned char *)malloc(n ? n : 1); }

static const uint64_t KEYS[] = {0, 1, 2, 0xFFFFFFFFFFFFFFFFull, 0x8000000000000000ull, 0x3A9F1B6E52C8D407ull,
                                0xB5AD4ECEDA1CE2A9ull, 0x0000000100000001ull};
static const uint64_t CTRS[] = {0, 1, 0xFFFFFFFFFFFFFFFFull, 0xFFFFFFFFFFFFFFFEull, 0x7FFFFFFFFFFFFFFFull,
                                0x0123456789ABCDEFull, 0x00000000FFFFFFFFull};
#define NK (sizeof KEYS / sizeof KEYS[0])
#define NC (sizeof CTRS / sizeof CTRS[0])

/* kind's output bytes at counter c (element i of a range from ctr0). */
static void element(int kind, uint64_t key, uint64_t ctr0, uint64_t i, unsigned char *dst)
{
    const int split = kind == 4 || kind == 5;
    const uint64_t c = ctr0 + (split ? i / 2 : i);
    switch (kind) {
    case 0: { uint32_t v = oracle_squares32(c, key); memcpy(dst, &v, 4); break; }
    case 1: { float v = oracle_to_f32(oracle_squares32(c, key)); memcpy(dst, &v, 4); break; }
    case 2: { uint64_t v = oracle_squares64(c, key); memcpy(dst, &v, 8); break; }
    case 3: { double v = oracle_to_f64(oracle_squares64(c, key)); memcpy(dst, &v, 8); break; }
    default: {
        uint64_t w = oracle_squares64(c, key);
        uint32_t h = (i % 2 == 0) ? (uint32_t)w : (uint32_t)(w >> 32);
        if (kind == 5) { float f = oracle_to_f32(h); memcpy(dst, &f, 4); }
        else memcpy(dst, &h, 4);
    }
    }
}

static void check_fills(void)
{
    static const uint64_t NS[] = {0, 1, 2, 3, 5, 64, 1000};
    for (int kind = 0; kind < 6; ++kind) {
        const int W = oracle_kind_bytes(kind);
        CHECK(W == 4 || W == 8, "kind %d bytes %d", kind, W);
        for (size_t k = 0; k < NK; ++k)
            for (size_t c = 0; c < NC; ++c)
                for (size_t t = 0; t < sizeof NS / sizeof NS[0]; ++t) {
                    const uint64_t n = NS[t];
                    unsigned char *a = exact(n * W), *b = exact(n * W), e[8];
                    CHECK(oracle_fill(kind, KEYS[k], CTRS[c], n, a) == 0, "fill kind %d", kind);
                    CHECK(oracle_fill_strided(kind, KEYS[k], CTRS[c], 1, n, b) == 0, "strided kind %d", kind);
                    CHECK(n == 0 || memcmp(a, b, n * W) == 0, "strided step 1 != fill, kind %d", kind);
                    for (uint64_t i = 0; i < n; ++i) {
                        element(kind, KEYS[k], CTRS[c], i, e);
                        if (memcmp(a + i * W, e, W) != 0) {
                            CHECK(0, "fill kind %d key %zu ctr %zu element %llu", kind, k, c, (unsigned long long)i);
                            break;
                        }
                    }
                    /* step 0 repeats the first counter; a huge step wraps */
                    CHECK(oracle_fill_strided(kind, KEYS[k], CTRS[c], 0, n, b) == 0, "step 0");
                    CHECK(oracle_fill_strided(kind, KEYS[k], CTRS[c], 0xFFFFFFFFFFFFFFFFull, n, b) == 0, "step -1");
                    free(a);
                    free(b);
                }
    }
    unsigned char one[8];
    CHECK(oracle_fill_strided(-1, 1, 0, 1, 1, one) != 0, "unknown kind accepted by strided fill");
    CHECK(oracle_kind_bytes(6) == 0 && oracle_kind_bytes(-1) == 0, "unknown kind has a width");
}

static void check_scalars(void)
{
    uint64_t ctrs[NK * NC], keys[NK * NC], tr[5], trb[5 * NK * NC];
    for (size_t k = 0; k < NK; ++k)
        for (size_t c = 0; c < NC; ++c) {
            ctrs[k * NC + c] = CTRS[c];
            keys[k * NC + c] = KEYS[k];
        }
    oracle_trace_batch(ctrs, keys, NK * NC, trb);
    for (size_t i = 0; i < NK * NC; ++i) {
        oracle_trace(ctrs[i], keys[i], tr);
        CHECK(memcmp(tr, trb + 5 * i, sizeof tr) == 0, "trace batch row %zu", i);
        CHECK((uint32_t)(oracle_squares64(ctrs[i], keys[i]) >> 32) == oracle_squares32(ctrs[i], keys[i]),
              "hi32(squares64) != squares32 at row %zu", i);
    }
    CHECK(oracle_to_f32(0) == 0.0f && oracle_to_f32(0xFFFFFFFFu) < 1.0f && oracle_to_f32(0xFFu) == 0.0f,
          "f32 edges");
    CHECK(oracle_to_f64(0) == 0.0 && oracle_to_f64(0xFFFFFFFFFFFFFFFFull) < 1.0 && oracle_to_f64(0x7FFull) == 0.0,
          "f64 edges");
}

static void check_keys(void)
{
    CHECK(oracle_key_index(0, 518918400ull) == 0, "index of 0");
    CHECK(oracle_key_index(0xFFFFFFFFFFFFFFFFull, 518918400ull) == 518918399ull, "index of 2^64-1");
    (void)oracle_key_upper(0);
    (void)oracle_key_upper(518918399ull);
    (void)oracle_key_lower(0);
    CHECK((oracle_key_lower(259459199ull) & 1u) == 1u, "lower half ends in an odd digit");
    static const uint64_t MS[] = {0, 1, 2, 257};
    for (size_t t = 0; t < sizeof MS / sizeof MS[0]; ++t) {
        const uint64_t m = MS[t];
        uint64_t *keys = (uint64_t *)exact(8 * m);
        CHECK(oracle_make_keys(0x243F6A8885A308D3ull, 0xFFFFFFFFFFFFFF00ull, m, keys) == 0, "make_keys");
        for (uint64_t j = 0; j < m; ++j) {
            int seen_hi = 0, seen_lo = 0;
            for (int d = 0; d < 8; ++d) {
                seen_hi |= 1 << (int)((keys[j] >> (32 + 4 * d)) & 15);
                seen_lo |= 1 << (int)((keys[j] >> (4 * d)) & 15);
            }
            CHECK(__builtin_popcount(seen_hi) == 8 && __builtin_popcount(seen_lo) == 8 && (keys[j] & 1),
                  "key %llu %016llx", (unsigned long long)j, (unsigned long long)keys[j]);
        }
        for (int kind = 0; kind < 4; ++kind) {
            const int W = oracle_kind_bytes(kind);
            unsigned char *out = exact(m * W), e[8];
            CHECK(oracle_fill_keys(kind, 0xFFFFFFFFFFFFFFFFull, keys, m, out) == 0, "fill_keys kind %d", kind);
            for (uint64_t j = 0; j < m; ++j) {
                element(kind, keys[j], 0xFFFFFFFFFFFFFFFFull, 0, e);
                CHECK(memcmp(out + j * W, e, W) == 0, "fill_keys kind %d key %llu", kind, (unsigned long long)j);
            }
            free(out);
        }
        unsigned char one[8];
        CHECK(m == 0 || oracle_fill_keys(4, 0, keys, 1, one) != 0, "split kind accepted by fill_keys");
        free(keys);
    }
}

static void check_batch_and_sums(void)
{
    /* streams of every kind, some empty, packed back to back at 4- or 8-byte
     * aligned offsets; the arena holds exactly their bytes */
    enum { M = 9 };
    uint64_t keys[M], ctr0s[M], lens[M], offs[M];
    uint8_t kinds[M];
    uint64_t at = 0;
    for (int s = 0; s < M; ++s) {
        kinds[s] = (uint8_t)(s % 6);
        keys[s] = KEYS[s % NK];
        ctr0s[s] = CTRS[s % NC];
        lens[s] = (uint64_t)(s * 37 % 11);
        const int W = oracle_kind_bytes(kinds[s]);
        const uint64_t A = kinds[s] < 2 ? 4 : 8;
        at = (at + A - 1) / A * A;
        offs[s] = at;
        at += lens[s] * W;
    }
    unsigned char *arena = exact(at);
    CHECK(oracle_fill_batch(M, keys, ctr0s, lens, offs, kinds, arena) == 0, "fill_batch");
    for (int s = 0; s < M; ++s) {
        const int W = oracle_kind_bytes(kinds[s]);
        unsigned char *ref = exact(lens[s] * W);
        oracle_fill(kinds[s], keys[s], ctr0s[s], lens[s], ref);
        CHECK(lens[s] == 0 || memcmp(arena + offs[s], ref, lens[s] * W) == 0, "batch stream %d", s);
        free(ref);
    }
    free(arena);
    uint8_t bad = 7;
    unsigned char one[8];
    uint64_t zero = 0, len1 = 1;
    CHECK(oracle_fill_batch(1, keys, ctr0s, &len1, &zero, &bad, one) != 0, "unknown kind accepted by fill_batch");

    for (int kind = 0; kind < 6; ++kind)
        for (size_t c = 0; c < NC; ++c) {
            const uint64_t n = 333;
            const int W = oracle_kind_bytes(kind);
            unsigned char *v = exact(n * W);
            uint64_t s[2];
            CHECK(oracle_sum(kind, KEYS[5], CTRS[c], n, s) == 0, "sum kind %d", kind);
            oracle_fill(kind == 1 ? 0 : kind == 3 ? 2 : kind == 5 ? 4 : kind, KEYS[5], CTRS[c], n, v);
            unsigned __int128 acc = 0;
            for (uint64_t i = 0; i < n; ++i) {
                if (W == 4) {
                    uint32_t x;
                    memcpy(&x, v + 4 * i, 4);
                    acc += (kind == 1 || kind == 5) ? (x >> 8) : x;
                } else {
                    uint64_t x;
                    memcpy(&x, v + 8 * i, 8);
                    acc += kind == 3 ? (x >> 11) : x;
                }
            }
            CHECK(s[0] == (uint64_t)acc && s[1] == (uint64_t)(acc >> 64), "sum kind %d ctr %zu", kind, c);
            free(v);
        }
    uint64_t s[2];
    CHECK(oracle_sum(6, 1, 0, 1, s) != 0, "unknown kind accepted by sum");
    CHECK(oracle_sum(0, 1, 0, 0, s) == 0 && s[0] == 0 && s[1] == 0, "empty sum");
}

int main(void)
{
    check_scalars();
    check_fills();
    check_keys();
    check_batch_and_sums();
    printf("%s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
