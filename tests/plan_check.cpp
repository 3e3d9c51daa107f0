// Test program (run on the CPU by tests/test_abi.py): the fill's launch
// plan keeps every launch below 2^32 work-items and 2^31 workgroups, covers
// the body's chunks exactly once and in order, and splits fills of 2^33
// 8-byte and 2^34 4-byte outputs (one 4 KiB chunk per workgroup) into more
// than one launch; the grids of key-counter mode and of the batch fill stay
// within the same limits at any size.  Host code only (sqi::plan_fill,
// sqi::keys_grid, sqi::batch_grid); no device is touched.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "../paper_2004_06278_amd/csrc/sq_internal.hpp"

static int failures = 0;

#define EXPECT(c, ...)                    \
  do {                                    \
    if (!(c)) {                           \
      ++failures;                         \
      printf("FAIL %s: ", #c);            \
      printf(__VA_ARGS__);                \
      printf("\n");                       \
    }                                     \
  } while (0)

static void check(const char* name, uint64_t nvec, sq_launch_cfg cfg, uint32_t cus, size_t want_min_segs) {
  std::vector<sqi::FillSegment> segs;
  sqi::plan_fill(nvec, cfg, cus, segs);
  const uint64_t per = (uint64_t)cfg.block * cfg.unroll;
  const uint64_t nchunks = (nvec + per - 1) / per;
  uint64_t next = 0, vecs = 0;
  for (size_t i = 0; i < segs.size(); ++i) {
    const sqi::FillSegment& g = segs[i];
    EXPECT(g.first_chunk == next, "%s segment %zu starts at %llu, expected %llu", name, i,
           (unsigned long long)g.first_chunk, (unsigned long long)next);
    EXPECT((uint64_t)g.grid * cfg.block < (1ull << 32), "%s segment %zu grid %u x block %u", name, i, g.grid,
           cfg.block);
    EXPECT(g.grid >= 1 && g.grid < (1u << 31), "%s segment %zu grid %u", name, i, g.grid);
    EXPECT(g.nchunks <= sqi::max_segment_chunks(cfg.block), "%s segment %zu has %u chunks", name, i, g.nchunks);
    if (g.xcd_map == 2) EXPECT(g.grid == g.nchunks || (g.nchunks == 0 && g.grid == 1), "%s one chunk per group", name);
    EXPECT(g.full <= g.nchunks && (g.rem == 0 || g.full + 1 == g.nchunks) && g.rem < per,
           "%s segment %zu full %u rem %u of %u", name, i, g.full, g.rem, g.nchunks);
    vecs += (uint64_t)g.full * per + g.rem;
    next += g.nchunks;
  }
  EXPECT(next == nchunks, "%s covers %llu of %llu chunks", name, (unsigned long long)next,
         (unsigned long long)nchunks);
  EXPECT(vecs == nvec, "%s covers %llu of %llu vectors", name, (unsigned long long)vecs, (unsigned long long)nvec);
  EXPECT(segs.size() >= want_min_segs, "%s: %zu launches", name, segs.size());
  printf("%-44s vectors %llu chunks %llu launches %zu\n", name, (unsigned long long)nvec,
         (unsigned long long)nchunks, segs.size());
}

static void check_grid(const char* name, uint32_t grid, uint32_t block, uint64_t want) {
  EXPECT((uint64_t)grid * block < (1ull << 32), "%s: grid %u x block %u", name, grid, block);
  EXPECT(grid >= 1 && grid < (1u << 31), "%s: grid %u", name, grid);
  if (want) EXPECT(grid == want, "%s: grid %u, expected %llu", name, grid, (unsigned long long)want);
  printf("%-44s grid %u x %u\n", name, grid, block);
}

int main() {
  const sq_launch_cfg one{256, 1, 1, 2, 16};     // one 4 KiB chunk per workgroup (the default)
  const sq_launch_cfg big{1024, 8, 1, 2, 16};    // 128 KiB chunks
  const sq_launch_cfg gs0{256, 4, 8, 0, 16};     // grid-stride
  const sq_launch_cfg gs1{256, 4, 8, 1, 16};     // XCD-contiguous
  // 16-byte vectors: 2^33 U64 outputs = 2^32 vectors, 2^34 U32 outputs = 2^32 vectors
  check("2^33 x 8 B, one chunk per workgroup", 1ull << 32, one, 256, 2);
  check("2^34 x 4 B, one chunk per workgroup", 1ull << 32, one, 256, 2);
  check("2^35 x 4 B + 3 vectors, one chunk per workgroup", (1ull << 33) + 3, one, 256, 3);
  check("2^32 x 4 B, one chunk per workgroup", 1ull << 30, one, 256, 1);
  check("2^32 + 2^30 x 8 B, one chunk per workgroup", (1ull << 31) + (1ull << 29), one, 256, 1);
  check("2^33 x 8 B, 1024 x 8 chunks", 1ull << 32, big, 256, 1);
  check("2^33 x 8 B + 1 vector, grid-stride", (1ull << 32) + 1, gs0, 256, 1);
  check("2^33 x 8 B, XCD-contiguous", 1ull << 32, gs1, 256, 1);
  check("small, XCD-contiguous below 8 groups", 3000, gs1, 256, 1);
  check("empty body (head and tail only)", 0, one, 256, 1);
  check("one partial chunk", 17, one, 256, 1);
  // key-counter mode: 2^33 U64 keys = 2^32 vectors of two outputs; 2^34 U32 keys = 2^32 vectors
  const sq_launch_cfg k1{256, 1, 1, 2, 16}, k2{1024, 1, 1, 2, 16}, kp{256, 1, 8, 0, 16}, k64{64, 1, 1, 2, 16};
  check_grid("keys 2^33 U64, one vector per lane", sqi::keys_grid(1ull << 32, k1, 256), 256, 0);
  check_grid("keys 2^34 U32, 1024 lanes", sqi::keys_grid(1ull << 32, k2, 256), 1024, 0);
  check_grid("keys 2^20 vectors, one vector per lane", sqi::keys_grid(1ull << 20, k1, 256), 256, 1u << 12);
  check_grid("keys 2^33 vectors, persistent", sqi::keys_grid(1ull << 33, kp, 256), 256, 256 * 8);
  check_grid("keys, no vector (tail only)", sqi::keys_grid(0, k1, 256), 256, 1);
  check_grid("keys 2^32 vectors, 64 lanes", sqi::keys_grid(1ull << 32, k64, 256), 64, 0xFFFFFFFFu / 64);
  // batch fill, one tile per workgroup: 2^23 tiles of 1024 lanes, 2^25 tiles of 256
  const sq_launch_cfg b1{1024, 8, 1, 2, 10}, b2{256, 8, 1, 2, 10}, bq{256, 8, 16, 1, 16};
  check_grid("batch 2^23 tiles x 1024 lanes", sqi::batch_grid(1ull << 23, b1, 256), 1024, 0);
  check_grid("batch 2^25 tiles x 256 lanes", sqi::batch_grid(1ull << 25, b2, 256), 256, 0xFFFFFFFFu / 256);
  check_grid("batch 1000 tiles, one per workgroup", sqi::batch_grid(1000, b2, 256), 256, 1000);
  check_grid("batch queue order", sqi::batch_grid(1ull << 30, bq, 256), 256, 256 * 16);
  printf("%s\n", failures ? "FAILED" : "ok");
  return failures ? 1 : 0;
}
