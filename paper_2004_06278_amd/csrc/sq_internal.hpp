// Internal interfaces shared by the library's translation units (kernels,
// C ABI, tuner, server).  Not installed; the public interface is squares.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/squares.h"

namespace sqi {

// ---------------------------------------------------------------- errors
int fail(int status, const std::string& msg);            // records msg, returns status
int fail_hip(hipError_t e, const char* what);            // SQ_EHIP with the HIP message
// Bytes per output element (0 for an unknown kind) and the alignment an
// output pointer or batch offset needs (split kinds write whole squares64
// outputs, so they need 8).
inline int kind_bytes(int kind) {
  switch (kind) {
    case SQ_U32: case SQ_F32: case SQ_U32X2: case SQ_F32X2: return 4;
    case SQ_U64: case SQ_F64: return 8;
    default: return 0;
  }
}
inline int kind_align(int kind) { return kind == SQ_U32 || kind == SQ_F32 ? 4 : (kind_bytes(kind) ? 8 : 0); }

// Nearest double (ties to even) of the 128-bit integer (hi:lo) times 2^e:
// the rounding the reduce applies to its exact sum, on the device in the
// final reduce kernel and on the host in sq_u128_to_double_scaled.  One
// rounding for every e: the bits dropped are those below the result's last
// place, which is 52 places under its leading bit, or 2^-1074 where the
// result is subnormal.
__host__ __device__ inline double round_scaled(uint64_t lo, uint64_t hi, int e) {
  if (hi == 0 && lo < (1ull << 53)) return ldexp((double)lo, e);  // exact, rounded once by ldexp
  // beyond these bounds every S in [2^53, 2^128) overflows or rounds to 0 alike
  if (e > 1100) e = 1100;
  if (e < -1300) e = -1300;
  const int msb = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
  int s = msb - 52;                  // bits dropped, >= 1
  if (s + e < -1074) s = -1074 - e;  // subnormal result: its last place is 2^-1074
  const unsigned __int128 S = ((unsigned __int128)hi << 64) | lo;
  if (s > msb) {  // S * 2^e is below one unit of the last place: that unit or 0
    const bool up = s == msb + 1 && S > (((unsigned __int128)1) << msb);  // above half; a tie goes to 0 (even)
    return up ? ldexp(1.0, s + e) : 0.0;
  }
  uint64_t mant = (uint64_t)(S >> s);
  const unsigned __int128 rem = S & ((((unsigned __int128)1) << s) - 1);
  const unsigned __int128 half = ((unsigned __int128)1) << (s - 1);
  if (rem > half || (rem == half && (mant & 1))) {
    ++mant;
    if (mant == (1ull << 53)) { mant >>= 1; ++s; }
  }
  return ldexp((double)mant, s + e);
}

// ---------------------------------------------------------------- device
struct DeviceInfo {
  int device = -1;
  int cus = 256;
  void* scratch = nullptr;               // this device's copy of the no-allocation reduce scratch
  hipError_t scratch_err = hipSuccess;   // why scratch is null, if it is
};
// Bytes of the file-scope device scratch that sq_reduce_noalloc uses in place
// of a caller's workspace (the reduce's 128-bit partials and queue counter).
constexpr size_t kNoAllocScratchBytes = 16ull * 65536 + 256;
int ensure_init();                 // binds device info for the current device
const DeviceInfo& device_info();

// ---------------------------------------------------------------- configs
bool cfg_valid(sq_op op, const sq_launch_cfg& c);
sq_launch_cfg default_cfg(sq_op op, int kind, uint64_t n);
sq_launch_cfg tuned_cfg(sq_op op, int kind, uint64_t n);  // table lookup (default if unset)

// ---------------------------------------------------------------- launches
// A fill's aligned body is written by one or more launches ("segments") of
// at most max_segment_chunks(block) chunks of block * unroll 16-byte
// vectors, so that chunk indices fit 32 bits and no grid reaches 2^32
// work-items.  plan_fill is host code (no device needed).
struct FillSegment {
  uint64_t first_chunk;  // index of the segment's first chunk in the body
  uint32_t nchunks;      // chunks in the segment
  uint32_t full;         // leading chunks that are whole
  uint32_t rem;          // vectors of the last chunk if it is not whole, else 0
  uint32_t grid;         // workgroups launched
  uint32_t xcd_map;      // chunk order actually used (1 falls back to 0 below 8 workgroups)
};
uint32_t max_segment_chunks(uint32_t block);
// The largest grid of `block`-lane workgroups below 2^32 work-items (and
// 2^31 workgroups), the launch limit the HIP headers state.  Host code, like the two grids below: key-counter mode
// over `work` vectors or keys (one per lane where the grid allows, else a
// grid-stride loop), and the batch fill over at most `tiles_bound` tiles
// (one per workgroup in order 2, else a persistent grid).
uint32_t grid_cap(uint32_t block);
uint32_t keys_grid(uint64_t work, const sq_launch_cfg& cfg, uint32_t cus);
uint32_t batch_grid(uint64_t tiles_bound, const sq_launch_cfg& cfg, uint32_t cus);
void plan_fill(uint64_t nvec, const sq_launch_cfg& cfg, uint32_t cus, std::vector<FillSegment>& segs);

// step: counter increment between consecutive outputs (1 for the plain
// fill and reduce).
hipError_t launch_fill(int kind, uint64_t key, uint64_t ctr0, uint64_t n, void* out,
                       const sq_launch_cfg& cfg, hipStream_t s, uint64_t step = 1);

constexpr uint32_t kReduceMaxParts = 65536;
hipError_t launch_reduce(int kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out,
                         void* ws, const sq_launch_cfg& cfg, hipStream_t s, uint64_t step = 1);
// Both sums of a pair over the same counters (kind32 SQ_U32 with SQ_U64, or
// SQ_F32 with SQ_F64) from one squares64 evaluation per counter; unit
// counter increments, queue order with chunks of 256 x 2^cfg.tile_log2.
hipError_t launch_reduce_pair(int kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out32,
                              sq_sum_result* out64, void* ws, const sq_launch_cfg& cfg, hipStream_t s);

// Key-counter mode: out[j] = kind's output at counter ctr under keys[j].
hipError_t launch_keys(int kind, uint64_t ctr, const uint64_t* keys, uint64_t m, void* out,
                       const sq_launch_cfg& cfg, hipStream_t s);

// squares32 and squares64 at one (ctr, key) into out[0], out[1] (device).
hipError_t launch_scalar(uint64_t ctr, uint64_t key, uint64_t* out, hipStream_t s);

// Distinct-digit keys from a counter range of squares64 under gen_key.
hipError_t launch_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t* keys,
                            const sq_launch_cfg& cfg, hipStream_t s);

// Descriptor arrays of a ragged batch (device pointers).
struct BatchDesc {
  const uint64_t* keys;
  const uint64_t* ctr0s;
  const uint64_t* lens;
  const uint64_t* offs;
  const uint8_t* kinds;
  uint32_t m;
  unsigned char* out;
  uint64_t out_bytes;
};

// Workspace header written by the tile scan; followed by tile_start[m+1]
// and the tile -> stream map.
struct BatchHdr {
  uint64_t total_tiles;
  uint32_t errors;
  uint32_t m;
  uint64_t next_tile;  // tile queue of the dynamic batch order (reset by the scan)
  uint64_t pad[5];
};
static_assert(sizeof(BatchHdr) == 64, "header is 64 bytes");
uint64_t batch_max_tiles(uint32_t m, uint64_t out_bytes);
size_t batch_ws_bytes(uint32_t m, uint64_t out_bytes);
hipError_t launch_batch(const BatchDesc& d, void* ws, const sq_launch_cfg& cfg, hipStream_t s);
// The batch kernels with the stream count read on the device from m_dev
// (nullptr: d.m), as a serving tick needs.
hipError_t launch_batch_body(const BatchDesc& d, const uint32_t* m_dev, void* ws, const sq_launch_cfg& cfg,
                             hipStream_t s);

// The autotuner's acceptance check: `run` writes a candidate's output into
// `buf` after `buf` was filled with a poison pattern (twice, two patterns);
// *same is true only if the first `bytes` bytes (a multiple of 4) equal
// `ref` both times, so a candidate that leaves any word unwritten fails.
// `bad` is a device counter of 8 bytes.
hipError_t tune_check_output(const void* ref, void* buf, uint64_t bytes, hipStream_t s, unsigned long long* bad,
                             const std::function<hipError_t()>& run, bool* same);

}  // namespace sqi
