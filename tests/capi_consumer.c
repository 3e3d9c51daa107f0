/* A plain C program that uses libsquares.so through include/squares.h only
 * (device memory from the HIP runtime's C API), checked against the CPU
 * oracle compiled into the same program.  TEST INFRASTRUCTURE: built by
 * __graft_entry__.build(), run by tests/test_gpu_capi.py on a GPU.
 * Exit status 0 when every check passes. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "squares.h"

/* oracle entry points (oracle/squares_oracle.c) */
void oracle_fill_u32(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out);
void oracle_fill_f64(uint64_t key, uint64_t ctr0, uint64_t n, double *out);
int oracle_sum(int kind, uint64_t key, uint64_t ctr0, uint64_t n, uint64_t out[2]);
int oracle_fill_batch(uint32_t m, const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                      const uint64_t *offs, const uint8_t *kinds, unsigned char *out);

static int failures = 0;
#define CHECK(cond, what)                                                        \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "FAIL %s (%s)\n", what, sq_last_error());            \
            ++failures;                                                          \
        }                                                                        \
    } while (0)
#define HIP(call)                                                                \
    do {                                                                         \
        if ((call) != hipSuccess) {                                              \
            fprintf(stderr, "HIP call failed: %s\n", #call);                     \
            return 2;                                                            \
        }                                                                        \
    } while (0)

int main(void)
{
    const uint64_t key = 0x9E3779B97F4A7C15ull, ctr0 = 0xFFFFFFFFFFFF0000ull;  /* wraps past 2^64 */
    const uint64_t n = (1u << 20) + 7;
    CHECK(sq_init() == SQ_OK, "sq_init");

    /* squares32 fill */
    uint32_t *d32 = NULL;
    HIP(hipMalloc((void **)&d32, n * sizeof *d32));
    CHECK(sq32_fill(key, ctr0, n, d32, NULL) == SQ_OK, "sq32_fill");
    uint32_t *h32 = malloc(n * sizeof *h32), *r32 = malloc(n * sizeof *r32);
    HIP(hipMemcpy(h32, d32, n * sizeof *h32, hipMemcpyDeviceToHost));
    oracle_fill_u32(key, ctr0, n, r32);
    CHECK(memcmp(h32, r32, n * sizeof *h32) == 0, "sq32_fill equals the oracle");

    /* uniform doubles */
    double *df = NULL;
    HIP(hipMalloc((void **)&df, n * sizeof *df));
    CHECK(sq_uniform_f64(key, ctr0, n, df, NULL) == SQ_OK, "sq_uniform_f64");
    double *hf = malloc(n * sizeof *hf), *rf = malloc(n * sizeof *rf);
    HIP(hipMemcpy(hf, df, n * sizeof *hf, hipMemcpyDeviceToHost));
    oracle_fill_f64(key, ctr0, n, rf);
    CHECK(memcmp(hf, rf, n * sizeof *hf) == 0, "sq_uniform_f64 equals the oracle");

    /* fused exact sum (F64 kind) */
    const size_t wsb = sq_reduce_workspace_bytes(n);
    void *ws = NULL;
    sq_sum_result *dres = NULL, hres;
    HIP(hipMalloc(&ws, wsb));
    HIP(hipMalloc((void **)&dres, sizeof *dres));
    CHECK(sq_reduce(SQ_F64, key, ctr0, n, dres, ws, wsb, NULL) == SQ_OK, "sq_reduce");
    HIP(hipMemcpy(&hres, dres, sizeof hres, hipMemcpyDeviceToHost));
    uint64_t ref[2];
    oracle_sum(3, key, ctr0, n, ref);
    CHECK(hres.lo == ref[0] && hres.hi == ref[1] && hres.n == n, "sq_reduce equals the oracle's exact sum");
    CHECK(sq_u128_to_double_scaled(ref[0], ref[1], -53) == hres.value, "nearest-even value");

    /* both widths in one pass (F32 and F64 sums) */
    sq_sum_result *dres2 = NULL, h32res, h64res;
    HIP(hipMalloc((void **)&dres2, 2 * sizeof *dres2));
    CHECK(sq_reduce_pair(SQ_F32, key, ctr0, n, dres2, dres2 + 1, ws, wsb, NULL) == SQ_OK, "sq_reduce_pair");
    HIP(hipMemcpy(&h32res, dres2, sizeof h32res, hipMemcpyDeviceToHost));
    HIP(hipMemcpy(&h64res, dres2 + 1, sizeof h64res, hipMemcpyDeviceToHost));
    uint64_t ref32[2];
    oracle_sum(1, key, ctr0, n, ref32);
    CHECK(h32res.lo == ref32[0] && h32res.hi == ref32[1], "paired F32 sum equals the oracle");
    CHECK(h64res.lo == ref[0] && h64res.hi == ref[1] && h64res.value == hres.value, "paired F64 sum equals sq_reduce");

    /* ragged batch: three streams of different kinds in one arena */
    const uint32_t m = 3;
    uint64_t keys[3] = {key, key + 2, 0x1234567890ABCDEFull};
    uint64_t ctrs[3] = {0, ctr0, 12345};
    uint64_t lens[3] = {5000, 70001, 1};
    uint64_t offs[3] = {0, 20000, 20000 + 8 * 70001};
    uint8_t kinds[3] = {SQ_U32, SQ_U64, SQ_F32};
    const uint64_t arena = offs[2] + 4 * lens[2];
    void *dk, *dc, *dl, *doff, *dkind, *dout, *bws;
    HIP(hipMalloc(&dk, sizeof keys));
    HIP(hipMalloc(&dc, sizeof ctrs));
    HIP(hipMalloc(&dl, sizeof lens));
    HIP(hipMalloc(&doff, sizeof offs));
    HIP(hipMalloc(&dkind, sizeof kinds));
    HIP(hipMalloc(&dout, arena));
    HIP(hipMemset(dout, 0, arena));
    const size_t bwsb = sq_batch_workspace_bytes(m, arena);
    HIP(hipMalloc(&bws, bwsb));
    HIP(hipMemcpy(dk, keys, sizeof keys, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dc, ctrs, sizeof ctrs, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dl, lens, sizeof lens, hipMemcpyHostToDevice));
    HIP(hipMemcpy(doff, offs, sizeof offs, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dkind, kinds, sizeof kinds, hipMemcpyHostToDevice));
    CHECK(sq_fill_batch(dk, dc, dl, doff, dkind, m, dout, arena, bws, bwsb, NULL) == SQ_OK, "sq_fill_batch");
    uint32_t errs = 99;
    CHECK(sq_batch_errors(bws, NULL, &errs) == SQ_OK && errs == 0, "no skipped streams");
    unsigned char *hb = malloc(arena), *rb = calloc(arena, 1);
    HIP(hipMemcpy(hb, dout, arena, hipMemcpyDeviceToHost));
    oracle_fill_batch(m, keys, ctrs, lens, offs, kinds, rb);
    CHECK(memcmp(hb, rb, arena) == 0, "sq_fill_batch equals the oracle");

    /* error paths never touch the device */
    CHECK(sq32_fill(key, ctr0, 10, NULL, NULL) == SQ_EINVAL, "null output rejected");
    CHECK(strlen(sq_last_error()) > 0, "error message set");
    CHECK(sq32_fill(key, ctr0, 10, (uint32_t *)((char *)d32 + 2), NULL) == SQ_EALIGN, "misaligned output rejected");

    hipFree(d32); hipFree(df); hipFree(ws); hipFree(dres); hipFree(dres2); hipFree(dk); hipFree(dc); hipFree(dl);
    hipFree(doff); hipFree(dkind); hipFree(dout); hipFree(bws);
    free(h32); free(r32); free(hf); free(rf); free(hb); free(rb);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("capi consumer: fill, uniform, reduce, paired reduce, batch and error paths match the oracle\n");
    return 0;
}
