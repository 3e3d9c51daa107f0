// Test program (run by tests/test_gpu_tune.py): the autotuner's acceptance
// check rejects candidates that leave part of the output unwritten and
// accepts ones that write every byte.  Links libsquares.so and calls the
// library's internal check (sqi::tune_check_output) with the library's own
// launchers; prints one line per case and exits non-zero on a wrong verdict.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "../paper_2004_06278_amd/csrc/sq_internal.hpp"

#define CK(x)                                                                                   \
  do {                                                                                          \
    hipError_t e_ = (x);                                                                        \
    if (e_ != hipSuccess) {                                                                     \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_));         \
      return 2;                                                                                 \
    }                                                                                           \
  } while (0)

static int failures = 0;

static void expect(const char* name, bool same, bool want) {
  printf("%-58s %s (expected %s)\n", name, same ? "accepted" : "rejected", want ? "accepted" : "rejected");
  if (same != want) ++failures;
}

int main() {
  using namespace sqi;
  if (ensure_init() != SQ_OK) {
    fprintf(stderr, "init failed: %s\n", sq_last_error());
    return 2;
  }
  const uint64_t key = 0x9B2F6E1D4C8A0357ull, ctr0 = 0xFFFFFFFFFFFF0000ull;
  const uint64_t n = (1ull << 20) + 3;  // U32 outputs, ragged
  void *ref = nullptr, *buf = nullptr, *ws = nullptr;
  unsigned long long* bad = nullptr;
  CK(hipMalloc(&ref, 4 * n + 64));
  CK(hipMalloc(&buf, 4 * n + 64));
  CK(hipMalloc(&ws, sq_reduce_workspace_bytes(n) + 64));
  CK(hipMalloc((void**)&bad, 8));
  hipStream_t s = nullptr;
  CK(hipStreamCreate(&s));
  const sq_launch_cfg def = default_cfg(SQ_OP_FILL, SQ_U32, n);
  const sq_launch_cfg other{64, 4, 1, 2, 16};
  const sq_launch_cfg gstride{256, 4, 4, 0, 16};
  CK(launch_fill(SQ_U32, key, ctr0, n, ref, def, s));
  bool same = false;
  CK(tune_check_output(ref, buf, 4 * n, s, bad, [&] { return launch_fill(SQ_U32, key, ctr0, n, buf, other, s); },
                       &same));
  expect("fill, another one-chunk-per-workgroup shape", same, true);
  CK(tune_check_output(ref, buf, 4 * n, s, bad, [&] { return launch_fill(SQ_U32, key, ctr0, n, buf, gstride, s); },
                       &same));
  expect("fill, grid-stride shape", same, true);
  CK(tune_check_output(ref, buf, 4 * n, s, bad,
                       [&] { return launch_fill(SQ_U32, key, ctr0, n - 1, buf, other, s); }, &same));
  expect("fill that skips the last output", same, false);
  CK(tune_check_output(ref, buf, 4 * n, s, bad,
                       [&] { return launch_fill(SQ_U32, key, ctr0 + 1, n - 1, (char*)buf + 4, other, s); },
                       &same));
  expect("fill that skips the first output", same, false);
  CK(tune_check_output(ref, buf, 4 * n, s, bad,
                       [&] { return launch_fill(SQ_U32, key, ctr0, n / 2, buf, other, s); }, &same));
  expect("fill that writes the first half only", same, false);
  // the old check: incumbent and candidate alternating in one buffer, the
  // candidate writing n - 1 outputs, compared without poison, passes
  CK(launch_fill(SQ_U32, key, ctr0, n, buf, def, s));
  CK(launch_fill(SQ_U32, key, ctr0, n - 1, buf, other, s));
  CK(hipStreamSynchronize(s));
  CK(tune_check_output(ref, buf, 4 * n, s, bad, [&] { return hipSuccess; }, &same));
  expect("a candidate that writes nothing", same, false);

  sq_sum_result* r_ref = (sq_sum_result*)ref;
  sq_sum_result* r_buf = (sq_sum_result*)buf;
  const sq_launch_cfg rdef = default_cfg(SQ_OP_REDUCE, SQ_F32, n);
  const sq_launch_cfg rother{256, 4, 4, 0, 16};
  CK(launch_reduce(SQ_F32, key, ctr0, n, r_ref, ws, rdef, s));
  CK(tune_check_output(r_ref, r_buf, sizeof(sq_sum_result), s, bad,
                       [&] { return launch_reduce(SQ_F32, key, ctr0, n, r_buf, ws, rother, s); }, &same));
  expect("reduce, static order", same, true);
  CK(tune_check_output(r_ref, r_buf, sizeof(sq_sum_result), s, bad, [&] { return hipSuccess; }, &same));
  expect("reduce that writes no result", same, false);
  CK(tune_check_output(r_ref, r_buf, sizeof(sq_sum_result), s, bad,
                       [&] { return launch_reduce(SQ_F32, key, ctr0, n - 1, r_buf, ws, rother, s); }, &same));
  expect("reduce over one counter less", same, false);
  CK(hipStreamSynchronize(s));
  printf("%s\n", failures ? "FAILED" : "ok");
  return failures ? 1 : 0;
}
