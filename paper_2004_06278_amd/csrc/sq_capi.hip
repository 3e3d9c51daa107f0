// C ABI of libsquares.so: argument checks, launch-configuration lookup and
// kernel launches for the fill, reduce and batch entry points declared in
// include/squares.h.  No generator arithmetic happens on the host.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "sq_internal.hpp"

namespace sqi {

static thread_local std::string g_err;

int fail(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

int fail_hip(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return SQ_EHIP;
}

// Scratch of sq_reduce_noalloc: the reduce's workspace as a file-scope
// device array, so that callers that cannot allocate (code under HIP graph
// capture, allocation-free serving loops) need no workspace.  Every device
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` only names the symbol: its device address, different on
// each device, comes from hipGetSymbolAddress (ensure_init, once per device)
// and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static_assert(kNoAllocScratchBytes == 16ull * kReduceMaxParts + 256, "scratch holds the reduce workspace");

static std::mutex g_dev_mu;
static std::unordered_map<int, DeviceInfo> g_devs;
static thread_local DeviceInfo t_cur;
int tune_autoload();  // sq_tune.cpp

int ensure_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  if (t_cur.device == dev) return SQ_OK;
  {
    std::lock_guard<std::mutex> g(g_dev_mu);
    auto it = g_devs.find(dev);
    if (it == g_devs.end()) {
      DeviceInfo di;
      di.device = dev;
      int cus = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute(CU count)");
      di.cus = cus > 0 ? cus : 256;
      // with `dev` current: this device's address of the scratch array
      void* p = nullptr;
      di.scratch_err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      di.scratch = di.scratch_err == hipSuccess ? p : nullptr;
      it = g_devs.emplace(dev, di).first;
    }
    t_cur = it->second;
  }
  return tune_autoload();
}

const DeviceInfo& device_info() { return t_cur; }

}  // namespace sqi

using namespace sqi;

#define SQ_INIT_OR_RETURN()          \
  do {                               \
    int rc_ = ensure_init();         \
    if (rc_ != SQ_OK) return rc_;    \
  } while (0)

extern "C" {

const char* sq_last_error(void) { return g_err.c_str(); }

int sq_version(void) { return 10100; }

int sq_init(void) {
  SQ_INIT_OR_RETURN();
  return SQ_OK;
}

// ---------------------------------------------------------------- fills
static int check_fill(int kind, uint64_t n, const void* out) {
  const int A = kind_align(kind);
  if (A == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string(kind));
  if (n == 0) return SQ_OK;
  if (out == nullptr) return fail(SQ_EINVAL, "null output pointer with n > 0");
  if (((uintptr_t)out & (uintptr_t)(A - 1)) != 0)
    return fail(SQ_EALIGN, "output pointer not aligned to " + std::to_string(A) + " bytes");
  return SQ_OK;
}

int sq_fill_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, void* out, const sq_launch_cfg* cfg,
                void* stream) {
  int rc = check_fill(kind, n, out);
  if (rc != SQ_OK || n == 0) return rc;
  if (cfg == nullptr || !cfg_valid(SQ_OP_FILL, *cfg)) return fail(SQ_EINVAL, "invalid fill launch configuration");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_fill(kind, key, ctr0, n, out, *cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "fill launch");
}

int sq_fill(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, void* out, void* stream) {
  int rc = check_fill(kind, n, out);
  if (rc != SQ_OK || n == 0) return rc;
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_FILL, kind, n);
  hipError_t e = launch_fill(kind, key, ctr0, n, out, cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "fill launch");
}

int sq32_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t* out, void* stream) {
  return sq_fill(SQ_U32, key, ctr0, n, out, stream);
}
int sq64_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint64_t* out, void* stream) {
  return sq_fill(SQ_U64, key, ctr0, n, out, stream);
}
int sq_uniform_f32(uint64_t key, uint64_t ctr0, uint64_t n, float* out, void* stream) {
  return sq_fill(SQ_F32, key, ctr0, n, out, stream);
}
int sq_uniform_f64(uint64_t key, uint64_t ctr0, uint64_t n, double* out, void* stream) {
  return sq_fill(SQ_F64, key, ctr0, n, out, stream);
}
int sq64x2_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t* out, void* stream) {
  return sq_fill(SQ_U32X2, key, ctr0, n, out, stream);
}
int sq_uniform_f32x2(uint64_t key, uint64_t ctr0, uint64_t n, float* out, void* stream) {
  return sq_fill(SQ_F32X2, key, ctr0, n, out, stream);
}

// ---------------------------------------------------------------- scalar evaluation
// One 16-byte device buffer per device, allocated on first use and kept.
static std::mutex g_scalar_mu;
static std::unordered_map<int, uint64_t*> g_scalar_buf;

static int scalar_eval(uint64_t ctr, uint64_t key, uint64_t out[2]) {
  SQ_INIT_OR_RETURN();
  std::lock_guard<std::mutex> g(g_scalar_mu);
  uint64_t*& buf = g_scalar_buf[device_info().device];
  hipError_t e = hipSuccess;
  if (buf == nullptr && (e = hipMalloc((void**)&buf, 256)) != hipSuccess) {
    buf = nullptr;
    return fail_hip(e, "scalar buffer allocation");
  }
  if ((e = launch_scalar(ctr, key, buf, nullptr)) != hipSuccess) return fail_hip(e, "scalar launch");
  if ((e = hipMemcpy(out, buf, 16, hipMemcpyDeviceToHost)) != hipSuccess) return fail_hip(e, "scalar copy");
  return SQ_OK;
}

int sq32_at(uint64_t ctr, uint64_t key, uint32_t* value) {
  if (value == nullptr) return fail(SQ_EINVAL, "null value pointer");
  uint64_t v[2];
  int rc = scalar_eval(ctr, key, v);
  if (rc == SQ_OK) *value = (uint32_t)v[0];
  return rc;
}

int sq64_at(uint64_t ctr, uint64_t key, uint64_t* value) {
  if (value == nullptr) return fail(SQ_EINVAL, "null value pointer");
  uint64_t v[2];
  int rc = scalar_eval(ctr, key, v);
  if (rc == SQ_OK) *value = v[1];
  return rc;
}

double sq_u128_to_double_scaled(uint64_t lo, uint64_t hi, int pow2_exp) { return round_scaled(lo, hi, pow2_exp); }

// ---------------------------------------------------------------- counter increments other than one
int sq_fill_strided_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n, void* out,
                        const sq_launch_cfg* cfg, void* stream) {
  int rc = check_fill(kind, n, out);
  if (rc != SQ_OK || n == 0) return rc;
  if (cfg == nullptr || !cfg_valid(SQ_OP_FILL, *cfg)) return fail(SQ_EINVAL, "invalid fill launch configuration");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_fill(kind, key, ctr0, n, out, *cfg, (hipStream_t)stream, step);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "strided fill launch");
}

int sq_fill_strided(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n, void* out,
                    void* stream) {
  int rc = check_fill(kind, n, out);
  if (rc != SQ_OK || n == 0) return rc;
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_FILL, kind, n);
  return sq_fill_strided_cfg(kind, key, ctr0, step, n, out, &cfg, stream);
}

// ---------------------------------------------------------------- key-counter mode
// Measured on MI355X over 2^28 keys: one-wave workgroups, one 16-byte
// output vector per lane and one workgroup per 64 vectors (no grid-stride
// loop) move keys in and outputs out at 6.0-6.4 TB/s, above a plain device
// copy of the keys (5.0 TB/s).
static sq_launch_cfg keys_default_cfg() {
  sq_launch_cfg c{};
  c.block = 64;
  c.unroll = 4;  // unused
  c.grid_per_cu = 1;
  c.xcd_map = 2;
  c.tile_log2 = 16;
  return c;
}

int sq_fill_keys_cfg(sq_kind kind, uint64_t ctr, const uint64_t* keys, uint64_t m, void* out,
                     const sq_launch_cfg* cfg, void* stream) {
  if (kind != SQ_U32 && kind != SQ_F32 && kind != SQ_U64 && kind != SQ_F64)
    return fail(SQ_EINVAL, "key-counter mode takes kinds U32, F32, U64 and F64, not " + std::to_string((int)kind));
  if (m == 0) return SQ_OK;
  if (keys == nullptr || out == nullptr) return fail(SQ_EINVAL, "null keys or output pointer with m > 0");
  if (((uintptr_t)keys & 7) != 0) return fail(SQ_EALIGN, "keys must be 8-byte aligned");
  if (((uintptr_t)out & (uintptr_t)(kind_bytes(kind) - 1)) != 0)
    return fail(SQ_EALIGN, "output pointer not aligned to " + std::to_string(kind_bytes(kind)) + " bytes");
  if (cfg == nullptr || !cfg_valid(SQ_OP_FILL, *cfg)) return fail(SQ_EINVAL, "invalid launch configuration");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_keys(kind, ctr, keys, m, out, *cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "key-counter launch");
}

int sq_fill_keys(sq_kind kind, uint64_t ctr, const uint64_t* keys, uint64_t m, void* out, void* stream) {
  const sq_launch_cfg cfg = keys_default_cfg();
  return sq_fill_keys_cfg(kind, ctr, keys, m, out, &cfg, stream);
}

// ---------------------------------------------------------------- key generation
int sq_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t* keys, void* stream) {
  if (m == 0) return SQ_OK;
  if (keys == nullptr) return fail(SQ_EINVAL, "null keys pointer with m > 0");
  if (((uintptr_t)keys & 7) != 0) return fail(SQ_EALIGN, "keys must be 8-byte aligned");
  if (m > (1ull << 62)) return fail(SQ_EINVAL, "m > 2^62: key j uses counters ctr0 + 2j and ctr0 + 2j + 1");
  SQ_INIT_OR_RETURN();
  sq_launch_cfg cfg = keys_default_cfg();
  cfg.grid_per_cu = 16;  // a grid-stride launch of 256-lane workgroups (the kernel is VALU-bound)
  hipError_t e = launch_make_keys(gen_key, ctr0, m, keys, cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "key generation launch");
}

// ---------------------------------------------------------------- reduce
size_t sq_reduce_workspace_bytes(uint64_t n) {
  (void)n;
  return 16ull * kReduceMaxParts + 256;  // 128-bit partials, then the chunk queue counter
}

int sq_reduce_strided_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                          sq_sum_result* out, void* ws, size_t ws_bytes, const sq_launch_cfg* cfg, void* stream) {
  if (kind_bytes(kind) == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  if (out == nullptr || ws == nullptr) return fail(SQ_EINVAL, "null result or workspace pointer");
  if (((uintptr_t)out & 7) != 0 || ((uintptr_t)ws & 15) != 0)
    return fail(SQ_EALIGN, "result must be 8-byte and workspace 16-byte aligned");
  if (ws_bytes < sq_reduce_workspace_bytes(n))
    return fail(SQ_ENOMEM, "reduce workspace smaller than sq_reduce_workspace_bytes()");
  if (cfg == nullptr || !cfg_valid(SQ_OP_REDUCE, *cfg)) return fail(SQ_EINVAL, "invalid reduce launch configuration");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_reduce(kind, key, ctr0, n, out, ws, *cfg, (hipStream_t)stream, step);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "reduce launch");
}

int sq_reduce_strided(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n, sq_sum_result* out,
                      void* ws, size_t ws_bytes, void* stream) {
  if (kind_bytes(kind) == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_REDUCE, kind, n);
  return sq_reduce_strided_cfg(kind, key, ctr0, step, n, out, ws, ws_bytes, &cfg, stream);
}

int sq_reduce_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out, void* ws,
                  size_t ws_bytes, const sq_launch_cfg* cfg, void* stream) {
  if (kind_bytes(kind) == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  if (out == nullptr || ws == nullptr) return fail(SQ_EINVAL, "null result or workspace pointer");
  if (((uintptr_t)out & 7) != 0 || ((uintptr_t)ws & 15) != 0)
    return fail(SQ_EALIGN, "result must be 8-byte and workspace 16-byte aligned");
  if (ws_bytes < sq_reduce_workspace_bytes(n))
    return fail(SQ_ENOMEM, "reduce workspace smaller than sq_reduce_workspace_bytes()");
  if (cfg == nullptr || !cfg_valid(SQ_OP_REDUCE, *cfg)) return fail(SQ_EINVAL, "invalid reduce launch configuration");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_reduce(kind, key, ctr0, n, out, ws, *cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "reduce launch");
}

int sq_reduce(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out, void* ws, size_t ws_bytes,
              void* stream) {
  if (kind_bytes(kind) == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_REDUCE, kind, n);
  return sq_reduce_cfg(kind, key, ctr0, n, out, ws, ws_bytes, &cfg, stream);
}

// The reduce on the library's file-scope scratch instead of a workspace
// argument: no allocation anywhere on this path (sq_reduce_workspace_bytes
// does not grow with n, so every n fits the fixed scratch).  The queue
// counter in it is reset by a kernel at the start of each call, and every
// partial that the final kernel reads is written by the same call.  Calls
// that overlap on one device share the scratch and race.
int sq_reduce_noalloc(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out, void* stream) {
  if (kind_bytes(kind) == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  SQ_INIT_OR_RETURN();
  const DeviceInfo& di = device_info();
  if (di.scratch == nullptr) return fail_hip(di.scratch_err, "hipGetSymbolAddress(scratch) of sq_reduce_noalloc");
  if (sq_reduce_workspace_bytes(n) > kNoAllocScratchBytes)
    return fail(SQ_ENOMEM, "reduce workspace of " + std::to_string(sq_reduce_workspace_bytes(n)) +
                               " bytes exceeds the no-allocation scratch of " + std::to_string(kNoAllocScratchBytes) +
                               " bytes");
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_REDUCE, kind, n);
  return sq_reduce_cfg(kind, key, ctr0, n, out, di.scratch, kNoAllocScratchBytes, &cfg, stream);
}

// ---------------------------------------------------------------- paired sums
int sq_reduce_pair_cfg(sq_kind kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out32,
                       sq_sum_result* out64, void* ws, size_t ws_bytes, const sq_launch_cfg* cfg, void* stream) {
  if (kind32 != SQ_U32 && kind32 != SQ_F32)
    return fail(SQ_EINVAL, "sq_reduce_pair takes SQ_U32 (paired with SQ_U64) or SQ_F32 (paired with SQ_F64), not " +
                               std::to_string((int)kind32));
  if (out32 == nullptr || out64 == nullptr || ws == nullptr) return fail(SQ_EINVAL, "null result or workspace pointer");
  if (out32 == out64) return fail(SQ_EINVAL, "the two results must be distinct");
  if (((uintptr_t)out32 & 7) != 0 || ((uintptr_t)out64 & 7) != 0 || ((uintptr_t)ws & 15) != 0)
    return fail(SQ_EALIGN, "results must be 8-byte and workspace 16-byte aligned");
  if (ws_bytes < sq_reduce_workspace_bytes(n))
    return fail(SQ_ENOMEM, "reduce workspace smaller than sq_reduce_workspace_bytes()");
  if (cfg == nullptr || !cfg_valid(SQ_OP_REDUCE, *cfg) || cfg->xcd_map != 1)
    return fail(SQ_EINVAL, "invalid paired reduce launch configuration (queue order, xcd_map 1)");
  SQ_INIT_OR_RETURN();
  hipError_t e = launch_reduce_pair(kind32, key, ctr0, n, out32, out64, ws, *cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "paired reduce launch");
}

int sq_reduce_pair(sq_kind kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out32,
                   sq_sum_result* out64, void* ws, size_t ws_bytes, void* stream) {
  // the fused reduce's default shape: 256 lanes, 2 counters per unrolled
  // step, up to 8 resident workgroups per CU, chunks of 256 x 2^8 counters
  const sq_launch_cfg cfg{256, 2, 8, 1, 8};
  return sq_reduce_pair_cfg(kind32, key, ctr0, n, out32, out64, ws, ws_bytes, &cfg, stream);
}

// ---------------------------------------------------------------- batch
size_t sq_batch_workspace_bytes(uint32_t m, uint64_t out_bytes) { return batch_ws_bytes(m, out_bytes); }

static int check_batch(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens, const uint64_t* offs,
                       const uint8_t* kinds, uint32_t m, void* out, uint64_t out_bytes, void* ws, size_t ws_bytes) {
  if (m == 0) return SQ_OK;
  if (!keys || !ctr0s || !lens || !offs || !kinds || !out || !ws)
    return fail(SQ_EINVAL, "null descriptor, output or workspace pointer");
  if (((uintptr_t)keys | (uintptr_t)ctr0s | (uintptr_t)lens | (uintptr_t)offs) & 7)
    return fail(SQ_EALIGN, "descriptor arrays must be 8-byte aligned");
  if (((uintptr_t)out & 7) != 0 || ((uintptr_t)ws & 15) != 0)
    return fail(SQ_EALIGN, "arena must be 8-byte and workspace 16-byte aligned");
  if (ws_bytes < batch_ws_bytes(m, out_bytes))
    return fail(SQ_ENOMEM, "batch workspace smaller than sq_batch_workspace_bytes()");
  return SQ_OK;
}

static uint64_t mean_bucket_len(uint32_t m) {
  (void)m;
  return 1ull << 20;  // descriptors are on the device; tune by a typical stream length
}

// With $SQ_DEBUG_VALIDATE set (and not "0"), sq_fill_batch copies the
// descriptors to the host (synchronising the stream) and rejects a batch
// whose streams the kernels would skip or whose ranges overlap.
static bool debug_validate() {
  const char* e = std::getenv("SQ_DEBUG_VALIDATE");
  return e && *e && *e != '0';
}

static int validate_batch_on_host(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens,
                                  const uint64_t* offs, const uint8_t* kinds, uint32_t m, uint64_t out_bytes,
                                  hipStream_t s) {
  (void)keys;
  (void)ctr0s;
  std::vector<uint64_t> L(m), O(m);
  std::vector<uint8_t> K(m);
  hipError_t e = hipMemcpyAsync(L.data(), lens, 8ull * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(O.data(), offs, 8ull * m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(K.data(), kinds, m, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e, "descriptor copy for validation");
  std::vector<std::pair<uint64_t, uint64_t>> ranges;
  for (uint32_t i = 0; i < m; ++i) {
    const int W = kind_bytes(K[i]);
    if (W == 0) return fail(SQ_EINVAL, "stream " + std::to_string(i) + ": unknown kind");
    if (O[i] % (uint64_t)kind_align(K[i]) != 0)
      return fail(SQ_EALIGN, "stream " + std::to_string(i) + ": offset not aligned for its kind");
    if (O[i] > out_bytes || L[i] > (out_bytes - O[i]) / (uint64_t)W)
      return fail(SQ_EINVAL, "stream " + std::to_string(i) + ": range past the arena");
    if (L[i]) ranges.push_back({O[i], O[i] + L[i] * (uint64_t)W});
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second)
      return fail(SQ_EINVAL, "streams overlap at byte " + std::to_string(ranges[i].first));
  return SQ_OK;
}

int sq_fill_batch_cfg(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens, const uint64_t* offs,
                      const uint8_t* kinds, uint32_t m, void* out, uint64_t out_bytes, void* ws, size_t ws_bytes,
                      const sq_launch_cfg* cfg, void* stream) {
  int rc = check_batch(keys, ctr0s, lens, offs, kinds, m, out, out_bytes, ws, ws_bytes);
  if (rc != SQ_OK || m == 0) return rc;
  if (cfg == nullptr || !cfg_valid(SQ_OP_BATCH, *cfg)) return fail(SQ_EINVAL, "invalid batch launch configuration");
  SQ_INIT_OR_RETURN();
  if (debug_validate()) {
    rc = validate_batch_on_host(keys, ctr0s, lens, offs, kinds, m, out_bytes, (hipStream_t)stream);
    if (rc != SQ_OK) return rc;
  }
  BatchDesc d{keys, ctr0s, lens, offs, kinds, m, (unsigned char*)out, out_bytes};
  hipError_t e = launch_batch(d, ws, *cfg, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "batch launch");
}

int sq_fill_batch(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens, const uint64_t* offs,
                  const uint8_t* kinds, uint32_t m, void* out, uint64_t out_bytes, void* ws, size_t ws_bytes,
                  void* stream) {
  int rc = check_batch(keys, ctr0s, lens, offs, kinds, m, out, out_bytes, ws, ws_bytes);
  if (rc != SQ_OK || m == 0) return rc;
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg cfg = tuned_cfg(SQ_OP_BATCH, SQ_U32, mean_bucket_len(m));
  return sq_fill_batch_cfg(keys, ctr0s, lens, offs, kinds, m, out, out_bytes, ws, ws_bytes, &cfg, stream);
}

int sq_fill_streams(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens, const uint64_t* offs,
                    const uint8_t* kinds, uint32_t m, void* out, uint64_t out_bytes, void* stream) {
  if (m == 0) return SQ_OK;
  if (!keys || !ctr0s || !lens || !offs || !kinds || !out) return fail(SQ_EINVAL, "null host descriptor or arena");
  for (uint32_t s = 0; s < m; ++s) {
    const int W = kind_bytes(kinds[s]), A = kind_align(kinds[s]);
    if (W == 0) return fail(SQ_EINVAL, "stream " + std::to_string(s) + ": unknown kind");
    if (offs[s] % A != 0 || ((uintptr_t)out & (uintptr_t)(A - 1)) != 0)
      return fail(SQ_EALIGN, "stream " + std::to_string(s) + ": misaligned offset");
    if (offs[s] > out_bytes || lens[s] > (out_bytes - offs[s]) / W)
      return fail(SQ_EINVAL, "stream " + std::to_string(s) + ": range past the arena");
  }
  SQ_INIT_OR_RETURN();
  for (uint32_t s = 0; s < m; ++s) {
    if (lens[s] == 0) continue;
    const sq_launch_cfg cfg = tuned_cfg(SQ_OP_FILL, kinds[s], lens[s]);
    hipError_t e = launch_fill(kinds[s], keys[s], ctr0s[s], lens[s], (unsigned char*)out + offs[s], cfg,
                               (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "fill launch");
  }
  return SQ_OK;
}

int sq_batch_errors(const void* ws, void* stream, uint32_t* count) {
  if (ws == nullptr || count == nullptr) return fail(SQ_EINVAL, "null workspace or count pointer");
  SQ_INIT_OR_RETURN();
  const BatchHdr* h = (const BatchHdr*)ws;
  uint32_t v = 0;
  hipError_t e = hipMemcpyAsync(&v, &h->errors, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "reading batch error count");
  *count = v;
  return SQ_OK;
}

// ---------------------------------------------------------------- batch plan (HIP graph)
struct sq_batch_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
};

int sq_batch_plan_create(const uint64_t* keys, const uint64_t* ctr0s, const uint64_t* lens, const uint64_t* offs,
                         const uint8_t* kinds, uint32_t m, void* out, uint64_t out_bytes, void* ws, size_t ws_bytes,
                         const sq_launch_cfg* cfg, sq_batch_plan** plan) {
  if (plan == nullptr) return fail(SQ_EINVAL, "null plan pointer");
  *plan = nullptr;
  if (m == 0) return fail(SQ_EINVAL, "a plan needs m > 0");
  int rc = check_batch(keys, ctr0s, lens, offs, kinds, m, out, out_bytes, ws, ws_bytes);
  if (rc != SQ_OK) return rc;
  SQ_INIT_OR_RETURN();
  const sq_launch_cfg c = cfg ? *cfg : tuned_cfg(SQ_OP_BATCH, SQ_U32, mean_bucket_len(m));
  if (!cfg_valid(SQ_OP_BATCH, c)) return fail(SQ_EINVAL, "invalid batch launch configuration");
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return fail_hip(e, "hipStreamCreate for capture");
  sq_batch_plan* p = new sq_batch_plan();
  p->device = device_info().device;
  BatchDesc d{keys, ctr0s, lens, offs, kinds, m, (unsigned char*)out, out_bytes};
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch_batch(d, ws, c, cap);
    hipError_t ee = hipStreamEndCapture(cap, &p->graph);
    e = le != hipSuccess ? le : ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  hipError_t de = hipStreamDestroy(cap);
  if (e == hipSuccess) e = de;
  if (e != hipSuccess) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return fail_hip(e, "capturing the batch graph");
  }
  *plan = p;
  return SQ_OK;
}

int sq_batch_plan_launch(sq_batch_plan* plan, void* stream) {
  if (plan == nullptr || plan->exec == nullptr) return fail(SQ_ENOTFOUND, "null or destroyed plan");
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  return e == hipSuccess ? SQ_OK : fail_hip(e, "hipGraphLaunch");
}

int sq_batch_plan_destroy(sq_batch_plan* plan) {
  if (plan == nullptr) return SQ_OK;
  hipError_t e1 = plan->exec ? hipGraphExecDestroy(plan->exec) : hipSuccess;
  hipError_t e2 = plan->graph ? hipGraphDestroy(plan->graph) : hipSuccess;
  delete plan;
  if (e1 != hipSuccess) return fail_hip(e1, "hipGraphExecDestroy");
  if (e2 != hipSuccess) return fail_hip(e2, "hipGraphDestroy");
  return SQ_OK;
}

}  // extern "C"
