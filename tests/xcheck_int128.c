/*
 * Test-only second transcription of the rounds, for a consistency check of
 * the oracle's build: every product is formed in full as unsigned __int128
 * and explicitly truncated to 64 bits, every rotation is written with the
 * halves extracted and recombined.  Section 2 (squares32) and Section 5
 * (squares64) define the rounds; this file shares no code with the oracle or
 * the GPU library.  Row i of `out` receives the value right after round r's
 * half square (before its rotation), r = 1..5, as the oracle's trace does.
 */
#include <stdint.h>

typedef unsigned __int128 u128;

static uint64_t low64(u128 v) { return (uint64_t)(v & (u128)0xFFFFFFFFFFFFFFFFull); }

static uint64_t swap_halves(uint64_t v)
{
    uint64_t hi = v >> 32, lo = v & 0xFFFFFFFFull;
    return (lo << 32) | hi;
}

void xcheck_trace_batch(const uint64_t *ctrs, const uint64_t *keys, uint64_t m, uint64_t *out)
{
    for (uint64_t i = 0; i < m; ++i) {
        uint64_t y = low64((u128)ctrs[i] * keys[i]);
        uint64_t z = low64(((u128)ctrs[i] + 1) * keys[i]);
        uint64_t x = y;
        for (int r = 1; r <= 5; ++r) {
            uint64_t a = (r % 2 == 1) ? y : z;
            uint64_t v = low64((u128)x * x + a);
            out[5 * i + (r - 1)] = v;
            x = swap_halves(v);
        }
    }
}
