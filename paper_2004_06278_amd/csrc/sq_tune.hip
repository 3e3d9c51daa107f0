// Launch-configuration table and the autotuner.
//
// The table holds one sq_launch_cfg per (op, kind, size bucket).  The
// autotuner times every candidate configuration with HIP events on scratch
// buffers it allocates itself, and accepts a candidate only if its output is
// bit-identical to the default configuration's output (a device compare),
// so a tuned table can never change results.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "sq_internal.hpp"

namespace sqi {

static constexpr int kOps = 3, kKinds = 6, kBuckets = 5;

struct Entry {
  sq_launch_cfg cfg;
  bool set;
};
static std::mutex g_tab_mu;
static Entry g_tab[kOps][kKinds][kBuckets];
static bool g_autoloaded = false;

static int bucket_of(uint64_t n) {
  if (n < (1ull << 16)) return 0;
  if (n < (1ull << 20)) return 1;
  if (n < (1ull << 24)) return 2;
  if (n < (1ull << 28)) return 3;
  return 4;
}

static bool in(uint32_t v, std::initializer_list<uint32_t> set) {
  return std::find(set.begin(), set.end(), v) != set.end();
}

bool cfg_valid(sq_op op, const sq_launch_cfg& c) {
  if (c.grid_per_cu < 1 || c.grid_per_cu > 64) return false;
  switch (op) {
    case SQ_OP_FILL:
      return in(c.block, {64, 128, 256, 512, 1024}) && in(c.unroll, {1, 2, 4, 8}) && c.xcd_map <= 2;
    case SQ_OP_REDUCE:
      return in(c.unroll, {1, 2, 4}) && c.xcd_map <= 1 && (c.xcd_map == 0 || (c.tile_log2 >= 6 && c.tile_log2 <= 16));
    case SQ_OP_BATCH:
      return in(c.block, {64, 128, 256, 512, 1024}) && in(c.unroll, {1, 2, 4, 8}) && c.tile_log2 >= 10 &&
             c.tile_log2 <= 24 && c.xcd_map <= 2;
  }
  return false;
}

sq_launch_cfg default_cfg(sq_op op, int kind, uint64_t n) {
  (void)n;
  switch (op) {
    // One 4 KiB chunk per workgroup (grid = chunks), 256 lanes with one
    // 16-byte vector each: the fastest fill shape measured on MI355X both
    // back to back and right after a compute-bound kernel.  Small one-shot
    // chunks keep the write front narrow and let retiring workgroups be
    // replaced anywhere.
    case SQ_OP_FILL:
      (void)kind;
      return sq_launch_cfg{256, 1, 1, 2, 16};
    // resident grid taking chunks of 256 x 2^8 counters from the queue:
    // 4-6% faster than the static split on MI355X (no tail from the
    // slowest workgroups)
    case SQ_OP_REDUCE: return sq_launch_cfg{256, 2, 8, 1, 8};
    // a persistent grid of two 256-lane workgroups per CU taking tiles of
    // 2^16 outputs from the queue: the fastest ragged-batch shape measured
    // on MI355X (dynamic balance with few descriptor loads per byte)
    default: return sq_launch_cfg{256, 8, 2, 1, 16};
  }
}

sq_launch_cfg tuned_cfg(sq_op op, int kind, uint64_t n) {
  std::lock_guard<std::mutex> g(g_tab_mu);
  const Entry& e = g_tab[op][(kind >= 0 && kind < kKinds) ? kind : 0][bucket_of(n)];
  return e.set ? e.cfg : default_cfg(op, kind, n);
}

static int load_file(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SQ_ENOTFOUND, std::string("cannot open tuning table ") + path);
  char line[512];
  std::vector<std::pair<int, Entry>> rows;
  int op, kind, bucket;
  unsigned block, unroll, gpc, xcd, tile;
  while (std::fgets(line, sizeof line, f)) {
    if (std::sscanf(line,
                    " {\"op\": %d, \"kind\": %d, \"bucket\": %d, \"block\": %u, \"unroll\": %u, \"grid_per_cu\": %u, "
                    "\"xcd_map\": %u, \"tile_log2\": %u",
                    &op, &kind, &bucket, &block, &unroll, &gpc, &xcd, &tile) == 8) {
      if (op < 0 || op >= kOps || kind < 0 || kind >= kKinds || bucket < 0 || bucket >= kBuckets) continue;
      sq_launch_cfg c{block, unroll, gpc, xcd, tile};
      if (!cfg_valid((sq_op)op, c)) continue;
      rows.push_back({(op * kKinds + kind) * kBuckets + bucket, Entry{c, true}});
    }
  }
  std::fclose(f);
  std::lock_guard<std::mutex> g(g_tab_mu);
  for (auto& r : rows) (&g_tab[0][0][0])[r.first] = r.second;
  return SQ_OK;
}

int tune_autoload() {
  {
    std::lock_guard<std::mutex> g(g_tab_mu);
    if (g_autoloaded) return SQ_OK;
    g_autoloaded = true;
  }
  const char* p = std::getenv("SQ_TUNE_CACHE");
  if (p && *p) (void)load_file(p);  // a missing cache leaves the defaults
  return SQ_OK;
}

// ---------------------------------------------------------------- compare kernel
__global__ void k_count_diff(const uint32_t* a, const uint32_t* b, uint64_t words, unsigned long long* bad) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t G = (uint64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (; i < words; i += G) c += a[i] != b[i];
  if (c) atomicAdd(bad, c);
}

struct Scratch {
  void* a = nullptr;
  void* b = nullptr;
  void* ctx = nullptr;                // result and workspace of the context kernel
  unsigned long long* bad = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Scratch() {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (ctx) (void)hipFree(ctx);
    if (bad) (void)hipFree(bad);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  }
};

// Acceptance check of a candidate configuration.  The timed runs alternate
// the incumbent and the candidate in one buffer, so a candidate that left
// part of the range unwritten would show the incumbent's bytes there and
// pass a plain compare.  Here the candidate runs alone into the buffer after
// it has been filled with a poison pattern, twice, with two patterns that
// differ in every byte (0xA5..., 0x5A...): a word the candidate does not
// write keeps the poison in at least one run and differs from the
// reference.  `bytes` is a multiple of 4.
hipError_t tune_check_output(const void* ref, void* buf, uint64_t bytes, hipStream_t s, unsigned long long* bad,
                             const std::function<hipError_t()>& run, bool* same) {
  *same = false;
  for (const int poison : {0xA5, 0x5A}) {
    hipError_t e = hipMemsetAsync(buf, poison, bytes, s);
    if (e == hipSuccess) e = run();
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_diff, dim3(device_info().cus * 8), dim3(256), 0, s, (const uint32_t*)ref,
                       (const uint32_t*)buf, bytes / 4, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    unsigned long long h = 1;
    e = hipMemcpyAsync(&h, bad, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (h != 0) return hipSuccess;
  }
  *same = true;
  return hipSuccess;
}

// Times the incumbent and a candidate in alternation (reps pairs after one
// warm-up of each), so clock and thermal drift during tuning affect both
// alike; returns the median of each.
template <typename FA, typename FB>
static hipError_t time_pair(Scratch& S, FA inc, FB cand, int reps, float* ms_inc, float* ms_cand) {
  hipError_t e = inc();
  if (e == hipSuccess) e = cand();
  if (e != hipSuccess) return e;
  std::vector<float> a, b;
  for (int r = 0; r < reps; ++r) {
    for (int which = 0; which < 2; ++which) {
      if ((e = hipEventRecord(S.e0, S.s)) != hipSuccess) return e;
      if ((e = which == 0 ? inc() : cand()) != hipSuccess) return e;
      if ((e = hipEventRecord(S.e1, S.s)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(S.e1)) != hipSuccess) return e;
      float ms = 0;
      if ((e = hipEventElapsedTime(&ms, S.e0, S.e1)) != hipSuccess) return e;
      (which == 0 ? a : b).push_back(ms);
    }
  }
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  *ms_inc = a[a.size() / 2];
  *ms_cand = b[b.size() / 2];
  return hipSuccess;
}

// The same with a context: each timed launch follows an untimed run of
// `ctx` and is then repeated back to back, and each side scores the sum of
// its two medians.  The shader clock a launch meets depends on what ran
// before it (a compute-bound kernel leaves it high, a run of memory-bound
// launches lower), and on MI355X the best fill shape differs between the
// two: squares32 with 64 lanes x 4 vectors takes 2.62 ms back to back but
// 2.86 ms after a fused sum, 256 lanes x 1 vector 2.74 ms and 2.50 ms.
template <typename FA, typename FB, typename FC>
static hipError_t time_pair_ctx(Scratch& S, FA inc, FB cand, FC ctx, int reps, float* score_inc,
                                float* score_cand) {
  hipError_t e = inc();
  if (e == hipSuccess) e = cand();
  if (e != hipSuccess) return e;
  std::vector<float> t[2][2];  // [side][after ctx, back to back]
  for (int r = 0; r < reps; ++r) {
    for (int which = 0; which < 2; ++which) {
      if ((e = ctx()) != hipSuccess) return e;
      for (int k = 0; k < 2; ++k) {
        if ((e = hipEventRecord(S.e0, S.s)) != hipSuccess) return e;
        if ((e = which == 0 ? inc() : cand()) != hipSuccess) return e;
        if ((e = hipEventRecord(S.e1, S.s)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(S.e1)) != hipSuccess) return e;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, S.e0, S.e1)) != hipSuccess) return e;
        t[which][k].push_back(ms);
      }
    }
  }
  float score[2];
  for (int w = 0; w < 2; ++w) {
    score[w] = 0;
    for (int k = 0; k < 2; ++k) {
      std::sort(t[w][k].begin(), t[w][k].end());
      score[w] += t[w][k][t[w][k].size() / 2];
    }
  }
  *score_inc = score[0];
  *score_cand = score[1];
  return hipSuccess;
}

// Representative problem size of a size bucket: the middle of the bucket,
// and 2^32 outputs for the open-ended last one.
static uint64_t bucket_size(int b) { return b == kBuckets - 1 ? (1ull << 32) : (1ull << (4 * b + 14)); }

static bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("SQ_TUNE_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

static void report(const char* op, int kind, int bucket, uint64_t n, const sq_launch_cfg& c, float ms, bool same) {
  if (!verbose()) return;
  std::fprintf(stderr, "tune %s kind=%d bucket=%d n=%llu block=%u unroll=%u gpc=%u xcd=%u tile=%u ms=%.4f %s\n", op,
               kind, bucket, (unsigned long long)n, c.block, c.unroll, c.grid_per_cu, c.xcd_map, c.tile_log2, ms,
               same ? "" : "MISMATCH");
}

static void set_entry(int op, int kind, int bucket, const sq_launch_cfg& c) {
  std::lock_guard<std::mutex> g(g_tab_mu);
  g_tab[op][kind][bucket] = Entry{c, true};
}

// Deterministic generator for the tuner's own synthetic batch descriptors.
static uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace sqi

using namespace sqi;

extern "C" {

int sq_tune_get(sq_op op, sq_kind kind, uint64_t n, sq_launch_cfg* cfg) {
  if (cfg == nullptr || (int)op < 0 || (int)op >= kOps || kind_bytes(kind) == 0)
    return fail(SQ_EINVAL, "bad tune_get arguments");
  *cfg = tuned_cfg(op, kind, n);
  return SQ_OK;
}

int sq_tune_set(sq_op op, sq_kind kind, uint64_t n, const sq_launch_cfg* cfg) {
  if (cfg == nullptr || (int)op < 0 || (int)op >= kOps || kind_bytes(kind) == 0)
    return fail(SQ_EINVAL, "bad tune_set arguments");
  if (!cfg_valid(op, *cfg)) return fail(SQ_EINVAL, "invalid launch configuration");
  set_entry(op, kind, bucket_of(n), *cfg);
  return SQ_OK;
}

int sq_tune_load(const char* path) {
  if (path == nullptr) return fail(SQ_EINVAL, "null path");
  return load_file(path);
}

int sq_tune_save(const char* path) {
  if (path == nullptr) return fail(SQ_EINVAL, "null path");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SQ_EINVAL, std::string("cannot write ") + path);
  std::lock_guard<std::mutex> g(g_tab_mu);
  std::fprintf(f, "[\n");
  bool first = true;
  for (int op = 0; op < kOps; ++op)
    for (int k = 0; k < kKinds; ++k)
      for (int b = 0; b < kBuckets; ++b) {
        const Entry& e = g_tab[op][k][b];
        if (!e.set) continue;
        std::fprintf(f,
                     "%s {\"op\": %d, \"kind\": %d, \"bucket\": %d, \"block\": %u, \"unroll\": %u, \"grid_per_cu\": "
                     "%u, \"xcd_map\": %u, \"tile_log2\": %u}",
                     first ? "" : ",\n", op, k, b, e.cfg.block, e.cfg.unroll, e.cfg.grid_per_cu, e.cfg.xcd_map,
                     e.cfg.tile_log2);
        first = false;
      }
  std::fprintf(f, "\n]\n");
  std::fclose(f);
  return SQ_OK;
}

int sq_autotune(uint32_t op_mask, uint64_t max_bytes, const char* save_path) {
  int rc = ensure_init();
  if (rc != SQ_OK) return rc;
  const uint64_t half = std::max<uint64_t>(max_bytes / 2, 16ull << 20) & ~(uint64_t)0xFFFF;
  Scratch S;
  hipError_t e = hipMalloc(&S.a, half);
  if (e == hipSuccess) e = hipMalloc(&S.b, half);
  if (e == hipSuccess) e = hipMalloc((void**)&S.bad, 64);
  if (e == hipSuccess) e = hipMalloc(&S.ctx, 4096 + sq_reduce_workspace_bytes(0));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&S.e0);
  if (e == hipSuccess) e = hipEventCreate(&S.e1);
  if (e != hipSuccess) return fail_hip(e, "autotune scratch allocation");
  const uint64_t key = 0x9B2F6E1D4C8A0357ull, ctr0 = 0xFFFFFFFFFFFF0000ull;  // crosses 2^64 on purpose

  if (op_mask & (1u << SQ_OP_FILL)) {
    // context of every timed fill: a compute-bound fused F64 sum over 2^31
    // counters (about 1 ms), as when generation alternates with compute
    const sq_launch_cfg ctx_cfg = default_cfg(SQ_OP_REDUCE, SQ_F64, 1ull << 31);
    auto ctx = [&] {
      return launch_reduce(SQ_F64, key, ctr0, 1ull << 31, (sq_sum_result*)S.ctx, (unsigned char*)S.ctx + 4096,
                           ctx_cfg, S.s);
    };
    for (int kind = 0; kind < kKinds; ++kind) {
      const uint64_t W = kind_bytes(kind);
      for (int b = 0; b < kBuckets; ++b) {
        uint64_t n = std::min<uint64_t>(bucket_size(b), half / W);
        n -= 3;  // ragged: exercises the tail (the buffers are aligned, as for timing)
        const sq_launch_cfg ref = default_cfg(SQ_OP_FILL, kind, n);
        if ((e = launch_fill(kind, key, ctr0, n, (unsigned char*)S.b, ref, S.s)) != hipSuccess) break;
        std::swap(S.a, S.b);  // reference now in a
        // The default is the first incumbent.  Each candidate is timed in
        // alternation with the incumbent (after the context kernel and back
        // to back) and replaces it when its score is 2% lower (below timing
        // noise) and its bytes equal the reference's.
        sq_launch_cfg best_c = ref;
        // candidates: one chunk per workgroup for every block and unroll,
        // and the grid-stride orders for the larger shapes
        std::vector<sq_launch_cfg> cands;
        for (uint32_t blk : {64u, 128u, 256u, 512u, 1024u})
          for (uint32_t u : {1u, 2u, 4u, 8u}) cands.push_back(sq_launch_cfg{blk, u, 1, 2, 16});
        for (uint32_t blk : {256u, 1024u})
          for (uint32_t u : {4u, 8u})
            for (uint32_t g : {1u, 4u, 16u, 64u})
              for (uint32_t x : {0u, 1u}) cands.push_back(sq_launch_cfg{blk, u, g, x, 16});
        for (const sq_launch_cfg& c : cands) {
          float ms_inc = 0, ms = 0;
          const sq_launch_cfg inc = best_c;
          e = time_pair_ctx(
              S, [&] { return launch_fill(kind, key, ctr0, n, (unsigned char*)S.b, inc, S.s); },
              [&] { return launch_fill(kind, key, ctr0, n, (unsigned char*)S.b, c, S.s); }, ctx, 5, &ms_inc, &ms);
          if (e != hipSuccess) break;
          bool same = false;
          e = tune_check_output(S.a, S.b, n * W, S.s, S.bad,
                                [&] { return launch_fill(kind, key, ctr0, n, (unsigned char*)S.b, c, S.s); }, &same);
          if (e != hipSuccess) break;
          report("fill", kind, b, n, c, ms, same);
          if (same && ms < 0.98f * ms_inc) best_c = c;
        }
        if (e != hipSuccess) break;
        report("fill-chosen", kind, b, n, best_c, 0.f, true);
        set_entry(SQ_OP_FILL, kind, b, best_c);
      }
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess) return fail_hip(e, "autotune fill");
  }

  if (op_mask & (1u << SQ_OP_REDUCE)) {
    sq_sum_result* res = (sq_sum_result*)S.a;        // reference result
    sq_sum_result* cand = (sq_sum_result*)S.b;       // candidate result
    void* ws = (unsigned char*)S.b + 4096;
    for (int kind = 0; kind < kKinds && e == hipSuccess; ++kind) {
      for (int b = 0; b < kBuckets && e == hipSuccess; ++b) {
        const uint64_t n = bucket_size(b) - 5;
        const sq_launch_cfg ref = default_cfg(SQ_OP_REDUCE, kind, n);
        if ((e = launch_reduce(kind, key, ctr0, n, res, ws, ref, S.s)) != hipSuccess) break;
        sq_launch_cfg best_c = ref;
        std::vector<sq_launch_cfg> cands;
        for (uint32_t u : {1u, 2u, 4u})
          for (uint32_t g : {2u, 4u, 8u, 16u, 32u}) cands.push_back(sq_launch_cfg{256, u, g, 0, 16});
        for (uint32_t g : {4u, 8u, 16u})
          for (uint32_t pl : {8u, 10u, 12u}) cands.push_back(sq_launch_cfg{256, 4, g, 1, pl});
        for (const sq_launch_cfg& c : cands) {
          const sq_launch_cfg inc = best_c;
          float ms_inc = 0, ms = 0;
          e = time_pair(
              S, [&] { return launch_reduce(kind, key, ctr0, n, cand, ws, inc, S.s); },
              [&] { return launch_reduce(kind, key, ctr0, n, cand, ws, c, S.s); }, 5, &ms_inc, &ms);
          if (e != hipSuccess) break;
          bool same = false;
          e = tune_check_output(res, cand, sizeof(sq_sum_result), S.s, S.bad,
                                [&] { return launch_reduce(kind, key, ctr0, n, cand, ws, c, S.s); }, &same);
          if (e != hipSuccess) break;
          report("reduce", kind, b, n, c, ms, same);
          if (same && ms < 0.98f * ms_inc) best_c = c;
        }
        if (e == hipSuccess) {
          report("reduce-chosen", kind, b, n, best_c, 0.f, true);
          set_entry(SQ_OP_REDUCE, kind, b, best_c);
        }
      }
    }
    if (e != hipSuccess) return fail_hip(e, "autotune reduce");
  }

  if (op_mask & (1u << SQ_OP_BATCH)) {
    // Synthetic ragged batches: log-uniform lengths around each bucket,
    // all four kinds, packed back to back (8-byte aligned).
    for (int b = 0; b < kBuckets && e == hipSuccess; ++b) {
      // bucket 2 (the one sq_fill_batch uses) spans lengths 2^10 .. 2^24
      const double lo_e = std::max(4.0 * b + 2, 6.0), hi_e = 4.0 * b + 16;
      const uint64_t budget = half - (1ull << 20);
      std::vector<uint64_t> keys, ctrs, lens, offs;
      std::vector<uint8_t> kinds;
      uint64_t rng = 12345 + b, pos = 0;
      while (keys.size() < 4096) {
        const double u = (double)(splitmix(rng) >> 11) * 0x1p-53;
        const uint8_t kd = (uint8_t)(splitmix(rng) & 3);
        const uint64_t W = kd < 2 ? 4 : 8;
        // 4-byte streams of even length: every offset stays 8-byte aligned,
        // so the streams cover [0, pos) without gaps and the acceptance
        // check can compare the whole range
        const uint64_t len = std::max<uint64_t>((uint64_t)std::exp2(lo_e + (hi_e - lo_e) * u) & ~1ull, 2);
        if (pos + len * W > budget) break;
        keys.push_back(splitmix(rng));
        ctrs.push_back(splitmix(rng));
        lens.push_back(len);
        offs.push_back(pos);
        kinds.push_back(kd);
        pos += len * W;
      }
      const uint32_t m = (uint32_t)keys.size();
      if (m == 0) continue;
      // descriptors live in a's tail region (after the arena) in both buffers' roles:
      // the arena is [0, budget) of a/b, descriptors + workspace follow in a separate allocation
      void* desc = nullptr;
      const size_t dbytes = 33ull * m + 64 + batch_ws_bytes(m, budget) + 4096;
      if ((e = hipMalloc(&desc, dbytes)) != hipSuccess) break;
      uint64_t* dk = (uint64_t*)desc;
      uint64_t* dc = dk + m;
      uint64_t* dl = dc + m;
      uint64_t* dof = dl + m;
      uint8_t* dkd = (uint8_t*)(dof + m);
      void* ws = (void*)(((uintptr_t)(dkd + m) + 255) & ~(uintptr_t)255);
      e = hipMemcpy(dk, keys.data(), 8ull * m, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dc, ctrs.data(), 8ull * m, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dl, lens.data(), 8ull * m, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dof, offs.data(), 8ull * m, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(dkd, kinds.data(), m, hipMemcpyHostToDevice);
      const uint64_t used = (pos + 255) & ~255ull;
      if (e == hipSuccess) e = hipMemsetAsync(S.a, 0, used, S.s);
      if (e == hipSuccess) e = hipMemsetAsync(S.b, 0, used, S.s);
      const sq_launch_cfg ref = default_cfg(SQ_OP_BATCH, 0, 0);
      sq_launch_cfg best_c = ref;
      if (e == hipSuccess) {
        BatchDesc d{dk, dc, dl, dof, dkd, m, (unsigned char*)S.a, budget};
        e = launch_batch(d, ws, ref, S.s);
      }
      // candidates: one tile per workgroup with small tiles, and persistent
      // grids with larger ones
      std::vector<sq_launch_cfg> cands;
      for (uint32_t tl : {10u, 11u, 12u, 13u})
        for (uint32_t blk : {64u, 128u, 256u}) cands.push_back(sq_launch_cfg{blk, 8, 1, 2, tl});
      for (uint32_t tl : {14u, 16u, 18u})
        for (uint32_t blk : {256u, 1024u})
          for (uint32_t g : {2u, 4u, 8u, 16u}) cands.push_back(sq_launch_cfg{blk, 8, g, 0, tl});
      for (uint32_t tl : {14u, 15u, 16u, 17u, 18u})
        for (uint32_t blk : {64u, 256u, 512u})
          for (uint32_t g : {2u, 4u})
            for (uint32_t u : {2u, 8u}) cands.push_back(sq_launch_cfg{blk, u, g, 1, tl});
      for (const sq_launch_cfg& c : cands) {
        if (e != hipSuccess) break;
        const sq_launch_cfg inc = best_c;
        BatchDesc d{dk, dc, dl, dof, dkd, m, (unsigned char*)S.b, budget};
        float ms_inc = 0, ms = 0;
        e = time_pair(S, [&] { return launch_batch(d, ws, inc, S.s); },
                      [&] { return launch_batch(d, ws, c, S.s); }, 5, &ms_inc, &ms);
        if (e != hipSuccess) break;
        bool same = false;
        e = tune_check_output(S.a, S.b, pos, S.s, S.bad, [&] { return launch_batch(d, ws, c, S.s); }, &same);
        if (e != hipSuccess) break;
        report("batch", -1, b, pos, c, ms, same);
        if (same && ms < 0.98f * ms_inc) best_c = c;
      }
      if (e == hipSuccess) report("batch-chosen", -1, b, pos, best_c, 0.f, true);
      hipError_t fe = hipFree(desc);
      if (e == hipSuccess) e = fe;
      if (e == hipSuccess) {
        for (int k = 0; k < kKinds; ++k) set_entry(SQ_OP_BATCH, k, b, best_c);
      }
    }
    if (e != hipSuccess) return fail_hip(e, "autotune batch");
  }
  if (save_path) return sq_tune_save(save_path);
  return SQ_OK;
}

}  // extern "C"
