// gfx950 kernels of the Squares RNG: bulk fill (unit and other counter
// increments), fused exact reduce, ragged batch (tile scan, tile map and a
// tile-queue fill), key-counter mode and key generation.
//
// Every kernel is plain VALU integer code (no MFMA: nothing is a
// contraction).  Fills are bound by HBM write bandwidth: each lane produces
// 16 bytes (four 32-bit or two 64-bit outputs of consecutive counters) per
// global_store_dwordx4, so a wave writes 1 KiB contiguous per instruction,
// and a workgroup writes `block * unroll` such vectors per chunk (the
// fastest launch gives each workgroup one 4 KiB chunk).  The reduce writes
// nothing per element; it is bound by the VALU issue rate.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "sq_device.hpp"
#include "sq_internal.hpp"

using namespace sqd;

// Structured-buffer load and store (the LLVM intrinsics, declared under
// their own names): the address is the descriptor's base plus
// vindex * stride, so a lane index needs no address arithmetic.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ u32x2 buffer_load_idx_v2(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                    int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");
__device__ void buffer_store_idx_v4(u32x4 vdata, __amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                    int aux) __asm("llvm.amdgcn.struct.ptr.buffer.store.v4i32");

namespace {

// ============================================================== fill
// One launch covers one segment of the 1 KiB-aligned body: at most
// max_segment_chunks() chunks, so chunk indices fit 32 bits and a grid of
// one workgroup per chunk stays below 2^32 work-items.  Larger fills are
// split into several launches on the same stream.
struct FillArgs {
  uint64_t key;
  uint64_t ctr0;          // counter of element 0 (head and tail elements)
  unsigned char* out;     // address of element 0 (element-aligned)
  unsigned char* body;    // first 16-byte vector of this segment (1 KiB aligned)
  uint64_t step;          // counter increment between consecutive outputs
  uint64_t dkey;          // step * key: first-Weyl-term increment per counter visited
  uint64_t y_body;        // first Weyl term of the segment's first vector
  uint64_t ekey;          // Weyl step from one vector to the next (CPV * dkey)
  uint64_t body_nvec;     // full vectors of the whole body (where the tail starts)
  uint32_t nchunks;       // chunks of B*U vectors in this segment
  uint32_t full;          // leading chunks of the segment that are whole
  uint32_t rem;           // vectors of the last chunk when it is not whole
  uint32_t head;          // elements before the body (< 1024 / W)
  uint32_t tail;          // elements after the body's last full vector (0..3)
  uint32_t xcd_map;       // chunk order, see sq_launch_cfg
  uint32_t edges;         // this launch also writes the head and tail elements
  uint32_t pad;
};

// Elements before the body (up to the first 1 KiB boundary) and after its
// last full vector, one element store each, by workgroup 0 of the launch
// that carries them.
template <int K>
__device__ __forceinline__ void fill_edges(const FillArgs& a) {
  constexpr int W = Kind<K>::W, E = 16 / W;
  if (!a.edges || blockIdx.x != 0) return;
  for (uint32_t t = threadIdx.x; t < a.head + a.tail; t += blockDim.x) {
    const uint64_t i = t < a.head ? (uint64_t)t : a.head + a.body_nvec * E + (t - a.head);
    store_elem<K>(a.out + i * W, a.ctr0, i, a.key, a.step);
  }
}

// One 16-byte vector of the body: unit counter increments share each
// counter's second Weyl term with the next counter's first.
template <int K, bool S>
__device__ __forceinline__ u32x4 body_vec(const FillArgs& a, uint64_t y) {
  if constexpr (S) return gen_vec_strided<K>(y, a.key, a.dkey);
  else return gen_vec<K>(y, a.key);
}

// Chunk c of the segment covers vectors [c*B*U, (c+1)*B*U); lane tid writes
// vectors c*B*U + u*B + tid, u < U, so each store instruction of a wave
// covers 1 KiB contiguous and a workgroup's U stores cover B*U*16 bytes.
// y is the lane's first Weyl term for the chunk.  The chunk's base address
// is workgroup-uniform (scalar registers); the store adds the lane's 32-bit
// offset, so a vector costs no address arithmetic on the VALU.
template <int K, int U, bool S>
__device__ __forceinline__ void fill_chunk(const FillArgs& a, uint32_t c, uint64_t y) {
  const uint32_t B = blockDim.x, tid = threadIdx.x;
  unsigned char* base = a.body + (uint64_t)c * B * U * 16;
  const uint64_t ystep = (uint64_t)B * a.ekey;
  if (c < a.full) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      *(u32x4*)(base + (uint64_t)u * B * 16 + tid * 16u) = body_vec<K, S>(a, y);
      y += ystep;
      // one vector's chains at a time: keeps VGPR use low (occupancy hides
      // the latency of the dependent rounds better than interleaving)
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (tid + (uint32_t)u * B < a.rem) *(u32x4*)(base + (uint64_t)u * B * 16 + tid * 16u) = body_vec<K, S>(a, y);
      y += ystep;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int K, int U, bool S>
__global__ __launch_bounds__(1024) void k_fill(FillArgs a) {
  fill_edges<K>(a);
  const uint32_t tid = threadIdx.x;
  const uint64_t cw = (uint64_t)blockDim.x * U * a.ekey;  // Weyl step from one chunk to the next
  if (a.xcd_map == 2) {
    // one chunk per workgroup (grid = nchunks): workgroups retire and the
    // next ones start in dispatch order, so the chip writes one narrow
    // moving window of the output
    const uint32_t c = blockIdx.x;
    if (c < a.nchunks) fill_chunk<K, U, S>(a, c, lane_weyl(opaque_uniform(a.y_body + c * cw), a.ekey, tid));
    return;
  }
  // persistent grids: the lane's offset tid*ekey is computed once
  const uint64_t lane_y = lane_weyl(0, a.ekey, tid);
  if (a.xcd_map == 0) {
#pragma unroll 1
    for (uint32_t c = blockIdx.x; c < a.nchunks; c += gridDim.x)
      fill_chunk<K, U, S>(a, c, opaque(opaque_uniform(a.y_body + c * cw) + lane_y));
  } else {
    // Workgroups are dispatched round-robin over the 8 XCDs; give XCD r the
    // r-th contiguous eighth of the chunks (gridDim.x is a multiple of 8).
    const uint32_t r = blockIdx.x & 7u, local = blockIdx.x >> 3, gx = gridDim.x >> 3;
    const uint32_t per = (a.nchunks + 7) / 8;
    const uint32_t beg = r * per;
    const uint32_t end = beg + per < a.nchunks ? beg + per : a.nchunks;
#pragma unroll 1
    for (uint32_t c = beg + local; c < end; c += gx)
      fill_chunk<K, U, S>(a, c, opaque(opaque_uniform(a.y_body + c * cw) + lane_y));
  }
}

// The one-chunk shape with one vector per lane (the fastest fill launch:
// 256 lanes, one 16-byte vector each) in the fewest instructions.  Its lane
// setup, the first Weyl term yc + tid*ekey and the store address, would take
// five VALU instructions per lane, spread over only four (or two) outputs.
// Here the host puts tid*ekey for every lane into the kernel arguments; each
// lane reads its entry with one structured-buffer load (index = tid, no
// address arithmetic), issued first so that its latency overlaps the
// scalar set-up, and adds the chunk's term in one 64-bit add; the vector is
// written with a structured-buffer store whose index is tid again.  The
// store is the lane's last instruction, so no later instruction can
// overwrite its data registers before the store has read them.  The block
// size is a compile-time constant: read from the dispatch, it would put a
// scalar load in front of the table load.
constexpr uint32_t kLaneBlock = 256;
constexpr uint64_t kLaneMinVec = 1ull << 22;  // 64 MiB of output
struct FillLaneArgs {
  uint64_t lane[kLaneBlock];  // lane[t] = t * ekey; first, so it starts the argument segment
  FillArgs a;
};
static_assert(offsetof(FillLaneArgs, lane) == 0, "the lane table starts the kernel arguments");

// Word 3 of a buffer descriptor: 32-bit data format (any valid one serves
// untyped dword loads and stores).
constexpr int kRsrcWord3 = 0x00020000;

template <int K, bool S>
__global__ __launch_bounds__(kLaneBlock) void k_fill_lanes(FillLaneArgs t) {
  const uint32_t c = blockIdx.x, tid = threadIdx.x;
  // the kernel's only argument starts the kernel-argument segment
  const auto tab = __builtin_amdgcn_make_buffer_rsrc((void*)__builtin_amdgcn_kernarg_segment_ptr(), (short)8,
                                                     (int)kLaneBlock, kRsrcWord3);
  const u32x2 off = buffer_load_idx_v2(tab, (int)tid, 0, 0, 0);
  const FillArgs& a = t.a;
  fill_edges<K>(a);
  if (c >= a.nchunks) return;
  const uint64_t yc = opaque_uniform(a.y_body + c * ((uint64_t)kLaneBlock * a.ekey));
  const uint64_t y = yc + (((uint64_t)off.y << 32) | off.x);
  const auto out = __builtin_amdgcn_make_buffer_rsrc(a.body + (uint64_t)c * (kLaneBlock * 16), (short)16,
                                                     (int)kLaneBlock, kRsrcWord3);
  if (c < a.full) buffer_store_idx_v4(body_vec<K, S>(a, y), out, (int)tid, 0, 0, 0);
  else if (tid < a.rem) buffer_store_idx_v4(body_vec<K, S>(a, y), out, (int)tid, 0, 0, 0);
}

typedef void (*FillLanesKernel)(FillLaneArgs);
template <bool S>
FillLanesKernel fill_lanes_kernel(int kind) {
  switch (kind) {
    case SQ_U32: return k_fill_lanes<0, S>;
    case SQ_F32: return k_fill_lanes<1, S>;
    case SQ_U64: return k_fill_lanes<2, S>;
    case SQ_F64: return k_fill_lanes<3, S>;
    case SQ_U32X2: return k_fill_lanes<4, S>;
    default: return k_fill_lanes<5, S>;
  }
}

typedef void (*FillKernel)(FillArgs);
template <int K, bool S>
FillKernel fill_kernel_for(uint32_t unroll) {
  switch (unroll) {
    case 1: return k_fill<K, 1, S>;
    case 2: return k_fill<K, 2, S>;
    case 4: return k_fill<K, 4, S>;
    default: return k_fill<K, 8, S>;
  }
}

template <bool S>
FillKernel fill_kernel(int kind, uint32_t unroll) {
  switch (kind) {
    case SQ_U32: return fill_kernel_for<0, S>(unroll);
    case SQ_F32: return fill_kernel_for<1, S>(unroll);
    case SQ_U64: return fill_kernel_for<2, S>(unroll);
    case SQ_F64: return fill_kernel_for<3, S>(unroll);
    case SQ_U32X2: return fill_kernel_for<4, S>(unroll);
    default: return fill_kernel_for<5, S>(unroll);
  }
}

// ============================================================== reduce
struct ReduceArgs {
  uint64_t key;
  uint64_t ctr0;
  uint64_t dkey;         // step * key: first-Weyl-term increment per counter visited
  uint64_t y0;           // (ctr0 + per * step * thread) * key is y0 + thread * ythread
  uint64_t ythread;      // per * dkey
  uint64_t n;            // counters to sum (split kinds: pairs of outputs)
  uint64_t per;          // counters per thread (contiguous; per chunk in queue order)
  uint64_t* partials;    // 2 x u64 per workgroup
  unsigned long long* next;  // queue order: next chunk
  uint64_t nchunks;          // queue order: chunks of blockDim.x * per counters
};

// Advances the first Weyl term past the counter whose second term is z: by
// unit counter increments that is z itself, else y + step*key.
template <bool S>
__device__ __forceinline__ uint64_t next_y(uint64_t y, uint64_t z, uint64_t dkey) {
  if constexpr (S) return y + dkey;
  else return z;
}

__device__ __forceinline__ void add128(uint64_t& lo, uint64_t& hi, uint64_t v_lo, uint64_t v_hi) {
  const uint64_t s = lo + v_lo;
  hi += v_hi + (s < lo);
  lo = s;
}

__device__ __forceinline__ void wave_sum128(uint64_t& lo, uint64_t& hi) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t olo = __shfl_xor((unsigned long long)lo, off);
    const uint64_t ohi = __shfl_xor((unsigned long long)hi, off);
    add128(lo, hi, olo, ohi);
  }
}

// Sum of a workgroup's (lo, hi) pairs into thread 0 (LDS only for the
// combine across waves).
__device__ __forceinline__ void block_sum128(uint64_t& lo, uint64_t& hi) {
  __shared__ uint64_t s_lo[16], s_hi[16];
  wave_sum128(lo, hi);
  const uint32_t w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) { s_lo[w] = lo; s_hi[w] = hi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t i = 1; i < nw; ++i) add128(lo, hi, s_lo[i], s_hi[i]);
  }
}

// Each thread sums its own contiguous run of counters.  The integer terms
// are accumulated exactly: in 64 bits over runs short enough not to
// overflow (FLUSH terms), then into a 128-bit total.  Round 1 of every
// counter after the run's first comes from running differences along the
// run's Weyl terms (two 64-bit adds instead of a squaring; fd_const).
// Adds the integer terms of cnt consecutive counters, the first with Weyl
// term y, to the 128-bit (lo, hi).
template <int K, int U, bool S>
__device__ __forceinline__ void run_sum(uint64_t y, uint64_t cnt, uint64_t key, uint64_t dkey, uint64_t& lo,
                                        uint64_t& hi) {
  // Weyl step from one counter of the run to the next, and its differences
  const FdConst k = fd_const(opaque_uniform(S ? dkey : key));
  uint64_t r1 = square_plus(y, y), d = fd_diff(y, k);
  if constexpr (K == 2) {
    // 64-bit terms: a 64-bit partial plus a 32-bit count of its carries,
    // folded into the 128-bit total every 2^20 terms
    uint64_t i = 0;
    while (i < cnt) {
      // run lengths fit 32 bits: 32-bit loop control stays on the scalar
      // unit when cnt is uniform
      const uint32_t len = (uint32_t)(cnt - i < (1u << 20) ? cnt - i : (1u << 20));
      uint64_t s = 0;
      uint32_t carries = 0;
      uint32_t j = 0;
      for (; j + U <= len; j += U) {
        y = opaque(y);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t z = y + key;
          unsigned long long c;
          s = __builtin_addcll(s, sum_term_after1<K>(r1, y, z), 0ull, &c);
          carries += (uint32_t)c;
          r1 += d;
          d += k.dd;
          y = next_y<S>(y, z, dkey);
        }
      }
      for (; j < len; ++j) {
        const uint64_t z = y + key;
        unsigned long long c;
        s = __builtin_addcll(s, sum_term_after1<K>(r1, y, z), 0ull, &c);
        carries += (uint32_t)c;
        r1 += d;
        d += k.dd;
        y = next_y<S>(y, z, dkey);
      }
      add128(lo, hi, s, carries);
      i += len;
    }
  } else {
    // Terms < 2^53 (F64) and < 2^32 (U32) go into a 64-bit partial that is
    // flushed before it could overflow.  F32 terms are < 2^24, so 256 of them
    // fit a 32-bit partial: one 32-bit add per output instead of a 64-bit one.
    typedef typename std::conditional<K == 1, uint32_t, uint64_t>::type Part;
    // split kinds: < 2^33 (U32X2) or < 2^25 (F32X2) per counter
    constexpr uint64_t FLUSH = K == 3 ? 1024 : (K == 1 ? 256 : (1u << 20));
    uint64_t i = 0;
    while (i < cnt) {
      const uint32_t len = (uint32_t)(cnt - i < FLUSH ? cnt - i : FLUSH);
      Part s = 0;
      uint32_t j = 0;
      for (; j + U <= len; j += U) {
        // opaque: otherwise loop-strength reduction rewrites every unrolled
        // y as base + (j+u)*key with its own induction variable, plus a
        // separate 32-bit add for its low word
        y = opaque(y);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t z = y + key;
          s += (Part)sum_term_after1<K>(r1, y, z);
          r1 += d;
          d += k.dd;
          y = next_y<S>(y, z, dkey);
        }
      }
      for (; j < len; ++j) {
        const uint64_t z = y + key;
        s += (Part)sum_term_after1<K>(r1, y, z);
        r1 += d;
        d += k.dd;
        y = next_y<S>(y, z, dkey);
      }
      add128(lo, hi, (uint64_t)s, 0);
      i += len;
    }
  }
}

// Static order: thread t sums counters [t*per, (t+1)*per) of the range.
template <int K, int U, bool S>
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t cnt = 0;
  if (__umul64hi(t, a.per) == 0 && t * a.per < a.n) {
    const uint64_t begin = t * a.per;
    cnt = a.n - begin < a.per ? a.n - begin : a.per;
  }
  uint64_t lo = 0, hi = 0;
  // A workgroup whose threads all have full runs passes the uniform count, so
  // the loop control stays on the scalar unit.
  if (((uint64_t)blockIdx.x + 1) * blockDim.x * a.per <= a.n)
    run_sum<K, U, S>(a.y0 + t * a.ythread, a.per, a.key, a.dkey, lo, hi);
  else
    run_sum<K, U, S>(a.y0 + t * a.ythread, cnt, a.key, a.dkey, lo, hi);
  block_sum128(lo, hi);
  if (threadIdx.x == 0) {
    a.partials[2 * blockIdx.x] = lo;
    a.partials[2 * blockIdx.x + 1] = hi;
  }
}

// Queue order: a resident grid takes chunks of blockDim.x * per counters
// from a counter in the workspace (zeroed by k_reduce_reset just before), so
// workgroups that run faster take more chunks; thread t of chunk c sums
// counters [c*B*per + t*per, +per).  Exact integer sums, so the result does
// not depend on which workgroup took which chunk.
template <int K, int U, bool S>
__global__ __launch_bounds__(256) void k_reduce_queue(ReduceArgs a) {
  __shared__ uint64_t s_chunk;
  const uint64_t chunk = (uint64_t)blockDim.x * a.per;
  uint64_t lo = 0, hi = 0;
#pragma unroll 1
  while (true) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(a.next, 1ull);
    __syncthreads();
    const uint64_t c = wave_uniform(s_chunk);  // same chunk for the whole workgroup
    __syncthreads();  // every lane has read s_chunk before lane 0 overwrites it
    if (c >= a.nchunks) break;
    const uint64_t begin = c * chunk + (uint64_t)threadIdx.x * a.per;
    if ((c + 1) * chunk <= a.n) {
      // whole chunk in range: the uniform count keeps the loop control scalar
      run_sum<K, U, S>(a.y0 + begin * a.dkey, a.per, a.key, a.dkey, lo, hi);
    } else {
      const uint64_t cnt = begin < a.n ? (a.n - begin < a.per ? a.n - begin : a.per) : 0;
      run_sum<K, U, S>(a.y0 + begin * a.dkey, cnt, a.key, a.dkey, lo, hi);
    }
  }
  block_sum128(lo, hi);
  if (threadIdx.x == 0) {
    a.partials[2 * blockIdx.x] = lo;
    a.partials[2 * blockIdx.x + 1] = hi;
  }
}

// ============================================================== paired sums
// The 32-bit and the 64-bit sum over the same counters from one squares64
// evaluation per counter: squares32 at a counter is the high word of
// squares64 at it (both compute round 4's value t = x*x + z; squares32
// returns its high word, squares64 keeps t whole and XORs a value below 2^32
// into its low word).  P = 1: the F32 and F64 sums; P = 0: the U32 and U64
// sums.
template <int P>
__device__ __forceinline__ void pair_terms(uint64_t v, typename std::conditional<P == 1, uint32_t, uint64_t>::type& s32,
                                           uint64_t& s64, uint32_t& carries) {
  if constexpr (P == 1) {
    s32 += (uint32_t)(v >> 40);  // squares32 >> 8
    s64 += v >> 11;
  } else {
    s32 += v >> 32;
    unsigned long long c;
    s64 = __builtin_addcll(s64, v, 0ull, &c);
    carries += (uint32_t)c;
  }
}

template <int P, int U>
__device__ __forceinline__ void run_sum_pair(uint64_t y, uint64_t cnt, uint64_t key, uint64_t& lo32,
                                             uint64_t& hi32, uint64_t& lo64, uint64_t& hi64) {
  const FdConst k = fd_const(opaque_uniform(key));
  uint64_t r1 = square_plus(y, y), d = fd_diff(y, k);
  // F32 terms < 2^24: 256 fit a 32-bit partial; F64 terms < 2^53: 256 fit
  // 64 bits.  U32 terms < 2^32: 2^20 fit 64 bits; U64 terms count carries.
  constexpr uint32_t FLUSH = P == 1 ? 256u : (1u << 20);
  typedef typename std::conditional<P == 1, uint32_t, uint64_t>::type Part32;
  uint64_t i = 0;
  while (i < cnt) {
    const uint32_t len = (uint32_t)(cnt - i < FLUSH ? cnt - i : FLUSH);
    Part32 s32 = 0;
    uint64_t s64 = 0;
    uint32_t carries = 0;
    uint32_t j = 0;
    for (; j + U <= len; j += U) {
      y = opaque(y);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint64_t z = y + key;
        pair_terms<P>(sq64_after1(r1, y, z), s32, s64, carries);
        r1 += d;
        d += k.dd;
        y = z;
      }
    }
    for (; j < len; ++j) {
      const uint64_t z = y + key;
      pair_terms<P>(sq64_after1(r1, y, z), s32, s64, carries);
      r1 += d;
      d += k.dd;
      y = z;
    }
    add128(lo32, hi32, (uint64_t)s32, 0);
    add128(lo64, hi64, s64, carries);
    i += len;
  }
}

// Queue order as k_reduce_queue (unit counter increments); the 32-bit sum's
// partials go to a.partials, the 64-bit sum's to partials64.
template <int P, int U>
__global__ __launch_bounds__(256) void k_reduce_pair_queue(ReduceArgs a, uint64_t* partials64) {
  __shared__ uint64_t s_chunk;
  const uint64_t chunk = (uint64_t)blockDim.x * a.per;
  uint64_t lo32 = 0, hi32 = 0, lo64 = 0, hi64 = 0;
#pragma unroll 1
  while (true) {
    if (threadIdx.x == 0) s_chunk = atomicAdd(a.next, 1ull);
    __syncthreads();
    const uint64_t c = wave_uniform(s_chunk);
    __syncthreads();
    if (c >= a.nchunks) break;
    const uint64_t begin = c * chunk + (uint64_t)threadIdx.x * a.per;
    if ((c + 1) * chunk <= a.n) {
      run_sum_pair<P, U>(a.y0 + begin * a.key, a.per, a.key, lo32, hi32, lo64, hi64);
    } else {
      const uint64_t cnt = begin < a.n ? (a.n - begin < a.per ? a.n - begin : a.per) : 0;
      run_sum_pair<P, U>(a.y0 + begin * a.key, cnt, a.key, lo32, hi32, lo64, hi64);
    }
  }
  block_sum128(lo32, hi32);
  if (threadIdx.x == 0) {
    a.partials[2 * blockIdx.x] = lo32;
    a.partials[2 * blockIdx.x + 1] = hi32;
  }
  __syncthreads();  // thread 0 has read the first combine's LDS before it is reused
  block_sum128(lo64, hi64);
  if (threadIdx.x == 0) {
    partials64[2 * blockIdx.x] = lo64;
    partials64[2 * blockIdx.x + 1] = hi64;
  }
}

__global__ void k_reduce_reset(unsigned long long* next) {
  if (threadIdx.x == 0) *next = 0;
}

// Sums the workgroup partials.  For a split kind with an odd count, the
// last output (the low half of the counter after the last full pair, whose
// first Weyl term is y_tail) is added here (split_tail: 4 or 5, else 0).
__global__ __launch_bounds__(256) void k_reduce_final(const uint64_t* partials, uint32_t nparts, uint64_t n, int e,
                                                      int split_tail, uint64_t y_tail, uint64_t key,
                                                      sq_sum_result* out) {
  uint64_t lo = 0, hi = 0;
  for (uint32_t i = threadIdx.x; i < nparts; i += blockDim.x) add128(lo, hi, partials[2 * i], partials[2 * i + 1]);
  block_sum128(lo, hi);
  if (threadIdx.x == 0) {
    if (split_tail == 4) add128(lo, hi, split_lo_term<4>(y_tail, y_tail + key), 0);
    if (split_tail == 5) add128(lo, hi, split_lo_term<5>(y_tail, y_tail + key), 0);
    out->lo = lo;
    out->hi = hi;
    out->value = sqi::round_scaled(lo, hi, e);
    out->n = n;
  }
}

typedef void (*ReduceKernel)(ReduceArgs);
template <int K, bool S, bool Q>
ReduceKernel reduce_kernel_for(uint32_t unroll) {
  switch (unroll) {
    case 1: return Q ? k_reduce_queue<K, 1, S> : k_reduce<K, 1, S>;
    case 2: return Q ? k_reduce_queue<K, 2, S> : k_reduce<K, 2, S>;
    default: return Q ? k_reduce_queue<K, 4, S> : k_reduce<K, 4, S>;
  }
}

template <bool S, bool Q>
ReduceKernel reduce_kernel(int kind, uint32_t unroll) {
  switch (kind) {
    case SQ_U32: return reduce_kernel_for<0, S, Q>(unroll);
    case SQ_F32: return reduce_kernel_for<1, S, Q>(unroll);
    case SQ_U64: return reduce_kernel_for<2, S, Q>(unroll);
    case SQ_F64: return reduce_kernel_for<3, S, Q>(unroll);
    case SQ_U32X2: return reduce_kernel_for<4, S, Q>(unroll);
    default: return reduce_kernel_for<5, S, Q>(unroll);
  }
}

// ============================================================== batch
// Tiles of stream s under tile size 2^lg, or 0 (and *bad = 1) when the
// descriptor is invalid: unknown kind, offset not a multiple of the element
// size, or a range past the arena.
__device__ __forceinline__ uint64_t stream_tiles(const sqi::BatchDesc& d, uint32_t s, uint32_t lg, uint32_t* bad) {
  const uint32_t kind = d.kinds[s];
  const uint64_t len = d.lens[s], off = d.offs[s];
  const uint32_t W = (kind < 2 || kind > 3) ? 4u : 8u;  // element bytes
  const uint32_t A = kind < 2 ? 4u : 8u;                // offset alignment (split kinds: whole squares64)
  if (kind > 5 || (off & (A - 1)) != 0 || off > d.out_bytes || len > (d.out_bytes - off) / W) {
    *bad += 1;
    return 0;
  }
  const uint32_t lk = lg - (W == 8);  // tiles hold 2^lg * 4 bytes whatever the kind
  return (len >> lk) + ((len & ((1ull << lk) - 1)) != 0);
}

// One workgroup: exclusive scan of per-stream tile counts into ts[0..m],
// plus the total and the count of skipped streams in the header.  If the
// tiles would exceed the map's capacity (only possible when streams overlap,
// which the interface forbids) nothing is scheduled and every stream counts
// as skipped.
__global__ __launch_bounds__(1024) void k_batch_scan(sqi::BatchDesc d, const uint32_t* m_dev, uint32_t lg,
                                                     uint64_t max_tiles, sqi::BatchHdr* hdr, uint64_t* ts) {
  __shared__ uint64_t part[1024];
  __shared__ uint32_t errs;
  const uint32_t m = m_dev ? *m_dev : d.m;
  const uint32_t tid = threadIdx.x, B = blockDim.x;
  const uint64_t per = ((uint64_t)m + B - 1) / B;  // 64-bit: no wrap for m near 2^32
  const uint32_t b = (uint32_t)std::min<uint64_t>((uint64_t)tid * per, m);
  const uint32_t e = (uint32_t)std::min<uint64_t>((uint64_t)b + per, m);
  if (tid == 0) errs = 0;
  __syncthreads();
  uint64_t local = 0;
  uint32_t bad = 0;
  for (uint32_t s = b; s < e; ++s) local += stream_tiles(d, s, lg, &bad);
  part[tid] = local;
  if (bad) atomicAdd(&errs, bad);
  __syncthreads();
  for (uint32_t off = 1; off < B; off <<= 1) {
    const uint64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = tid ? part[tid - 1] : 0;
  uint32_t dummy = 0;
  for (uint32_t s = b; s < e; ++s) {
    ts[s] = run;
    run += stream_tiles(d, s, lg, &dummy);
  }
  if (tid == B - 1) {
    const bool fits = part[B - 1] <= max_tiles;
    ts[m] = part[B - 1];
    hdr->total_tiles = fits ? part[B - 1] : 0;
    hdr->m = m;
    hdr->errors = fits ? errs : m;
    hdr->next_tile = 0;
  }
}

// tile -> stream map: map[t] = the stream whose tiles include t (largest s
// with ts[s] <= t), one binary search per tile, all tiles in parallel.
__global__ __launch_bounds__(256) void k_batch_map(const sqi::BatchHdr* hdr, const uint64_t* ts, uint32_t* map) {
  const uint64_t total = hdr->total_tiles;
  const uint32_t m = hdr->m;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = m - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (ts[mid] <= t) lo = mid; else hi = mid - 1;
    }
    map[t] = lo;
  }
}

// Sixteen bytes of consecutive outputs of kind K from the first Weyl term
// y0 and round 1's running-difference state (r1, d) at y0 (fd_const of
// key): round 1 of the vector's later counters comes from r1 += d,
// d += 2*key*key instead of squarings.
template <int K>
__device__ __forceinline__ u32x4 gen_vec_fd(uint64_t y0, uint64_t key, uint64_t r1, uint64_t d, uint64_t dd) {
  u32x4 o;
  if constexpr (Kind<K>::CPV == 4) {
    const uint64_t y1 = y0 + key, y2 = y1 + key, y3 = y2 + key, y4 = y3 + key;
    const uint64_t r1b = r1 + d, d1 = d + dd, r1c = r1b + d1, r1d = r1c + (d1 + dd);
    uint32_t v[4];
    v[0] = sq32_after1(r1, y0, y1);
    v[1] = sq32_after1(r1b, y1, y2);
    v[2] = sq32_after1(r1c, y2, y3);
    v[3] = sq32_after1(r1d, y3, y4);
    if constexpr (K == 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = __float_as_uint(to_f32(v[j]));
    }
    o.x = v[0]; o.y = v[1]; o.z = v[2]; o.w = v[3];
  } else {
    const uint64_t y1 = y0 + key, y2 = y1 + key;
    uint64_t a = sq64_after1(r1, y0, y1), b = sq64_after1(r1 + d, y1, y2);
    if constexpr (K == 3) {
      a = (uint64_t)__double_as_longlong(to_f64(a));
      b = (uint64_t)__double_as_longlong(to_f64(b));
    }
    if constexpr (K == 5) {
      o.x = __float_as_uint(to_f32((uint32_t)a)); o.y = __float_as_uint(to_f32((uint32_t)(a >> 32)));
      o.z = __float_as_uint(to_f32((uint32_t)b)); o.w = __float_as_uint(to_f32((uint32_t)(b >> 32)));
    } else {
      o.x = (uint32_t)a; o.y = (uint32_t)(a >> 32);
      o.z = (uint32_t)b; o.w = (uint32_t)(b >> 32);
    }
  }
  return o;
}

// The workgroup fills `cnt` outputs of kind K from counter ctr at p
// (element-aligned, workgroup-uniform): a head up to the next 1 KiB boundary
// and a tail, element stores, and in between chunks of B*U 16-byte vectors
// laid out as in the plain fill (each store instruction of a wave covers one
// aligned KiB).  A tile holds at most 2^24 outputs, so its vector counts fit
// 32 bits.  Lane tid owns vectors tid, tid + B, tid + 2B, ...: their first
// Weyl terms are B*ekey apart, so the lane carries its Weyl term and round
// 1's running differences from one vector to the next (fd_const along the
// key within a vector, along B*ekey between the lane's vectors): per vector
// that is four 64-bit adds instead of the squarings of its first counter
// and one 64-bit multiply; the lane's state is set up once per tile.  The
// stores add the lane's 32-bit offset to the chunk's uniform address.
// Lanes 0..B-1 of the workgroup take part.
template <int K, int U>
__device__ __forceinline__ void fill_range(uint64_t key, uint64_t ctr, uint64_t cnt, unsigned char* p, uint32_t B) {
  constexpr int W = Kind<K>::W, E = 16 / W;
  const uint32_t tid = threadIdx.x;
  const uint32_t mis = (uint32_t)((uintptr_t)p & 1023u);
  uint32_t head = mis ? (1024u - mis) / W : 0;
  if (head > cnt) head = (uint32_t)cnt;
  const uint32_t nvec = (uint32_t)((cnt - head) / E);
  const uint32_t tail = (uint32_t)(cnt - head - (uint64_t)nvec * E);
  for (uint32_t t = tid; t < head + tail; t += B) {
    const uint64_t i = t < head ? t : head + (uint64_t)nvec * E + (t - head);
    store_elem<K>(p + i * W, ctr, i, key);
  }
  if (tid >= nvec) return;  // no vector for this lane (also covers nvec == 0)
  unsigned char* body = p + (uint64_t)head * W;
  const uint64_t ekey = (uint64_t)Kind<K>::CPV * key;
  const uint64_t ystep = (uint64_t)B * ekey;  // Weyl step from one of the lane's vectors to its next
  const uint64_t y_body = (ctr + elem_ctr<K>(head)) * key;  // head is even for split kinds
  // the lane's first vector, and round 1's differences along the key
  // (within a vector) and along ystep (from vector to vector); between
  // vectors the key difference itself moves by 2*key*ystep
  const FdConst kc = fd_const(opaque_uniform(key)), kv = fd_const(opaque_uniform(ystep));
  const uint64_t dmove = opaque_uniform(kc.s2 * ystep);
  uint64_t y = opaque(lane_weyl(y_body, ekey, tid));
  uint64_t r1 = square_plus(y, y), d = fd_diff(y, kc), D = fd_diff(y, kv);
  const uint32_t per_chunk = B * U;
#pragma unroll 1
  for (uint32_t c0 = 0; c0 < nvec; c0 += per_chunk) {
    unsigned char* base = body + (uint64_t)c0 * 16;
    if (c0 + per_chunk <= nvec) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        *(u32x4*)(base + (uint64_t)u * B * 16 + tid * 16u) = gen_vec_fd<K>(y, key, r1, d, kc.dd);
        y += ystep;
        r1 += D;
        D += kv.dd;
        d += dmove;
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      const uint32_t rem = nvec - c0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (tid + (uint32_t)u * B < rem)
          *(u32x4*)(base + (uint64_t)u * B * 16 + tid * 16u) = gen_vec_fd<K>(y, key, r1, d, kc.dd);
        y += ystep;
        r1 += D;
        D += kv.dd;
        d += dmove;
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// Where tile t writes: its stream is one load from the tile map.
struct TileDesc {
  uint64_t t;
  uint64_t key;
  uint64_t ctr;
  uint64_t cnt;
  unsigned char* p;
  uint32_t kind;
  uint32_t pad;
};

__device__ __forceinline__ TileDesc tile_desc(const sqi::BatchDesc& d, uint32_t lg, const uint64_t* ts,
                                              const uint32_t* map, uint64_t t) {
  TileDesc r;
  r.t = t;
  const uint32_t s = map[t];
  r.kind = d.kinds[s];
  const uint32_t lk = lg - (r.kind == 2 || r.kind == 3);  // 2^lk outputs of the kind = 2^lg * 4 bytes
  const uint64_t T = 1ull << lk;
  const uint64_t off = (t - ts[s]) << lk;
  const uint64_t len = d.lens[s];
  r.cnt = len - off < T ? len - off : T;
  const bool split = r.kind > 3;  // two elements per counter; tiles hold an even count
  r.key = d.keys[s];
  r.ctr = d.ctr0s[s] + (split ? off >> 1 : off);
  const uint64_t pos = d.offs[s] + off * ((r.kind == 2 || r.kind == 3) ? 8u : 4u);  // byte offset in the arena
  // the same tile for every lane: keep its description in scalar registers
  // so the tile's setup and loop control run on the scalar unit
  r.key = wave_uniform(r.key);
  r.ctr = wave_uniform(r.ctr);
  r.cnt = wave_uniform(r.cnt);
  // the byte offset, not the pointer, goes through readfirstlane, so the
  // pointer stays derived from the kernel argument and the stores remain
  // global_store (not flat_store)
  r.p = d.out + wave_uniform(pos);
  r.kind = __builtin_amdgcn_readfirstlane(r.kind);
  return r;
}

template <int U>
__device__ __forceinline__ void run_tile(const TileDesc& r, uint32_t B) {
  switch (r.kind) {
    case 0: fill_range<0, U>(r.key, r.ctr, r.cnt, r.p, B); break;
    case 1: fill_range<1, U>(r.key, r.ctr, r.cnt, r.p, B); break;
    case 2: fill_range<2, U>(r.key, r.ctr, r.cnt, r.p, B); break;
    case 3: fill_range<3, U>(r.key, r.ctr, r.cnt, r.p, B); break;
    case 4: fill_range<4, U>(r.key, r.ctr, r.cnt, r.p, B); break;
    default: fill_range<5, U>(r.key, r.ctr, r.cnt, r.p, B); break;
  }
}

template <int U>
__device__ __forceinline__ void batch_tile(const sqi::BatchDesc& d, uint32_t lg, const uint64_t* ts,
                                           const uint32_t* map, uint64_t t) {
  run_tile<U>(tile_desc(d, lg, ts, map, t), blockDim.x);
}

// order 0: workgroup g takes tiles g, g + grid, g + 2*grid, ..., so the
// workgroups running at any moment write neighbouring parts of the arena
// (with a grid as large as the tile bound, one tile each: order 2).
// order 1: a persistent grid takes tiles from a queue in tile order, so
// workgroups that finish early take more (the write front stays narrow and
// no workgroup idles while another still has a static share left).
template <int U>
__global__ __launch_bounds__(1024) void k_batch_fill(sqi::BatchDesc d, uint32_t lg, uint32_t order,
                                                     sqi::BatchHdr* hdr, const uint64_t* ts, const uint32_t* map) {
  const uint64_t total = hdr->total_tiles;
  if (order != 1) {
#pragma unroll 1
    for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) batch_tile<U>(d, lg, ts, map, t);
    return;
  }
  __shared__ uint64_t s_tile;
#pragma unroll 1
  while (true) {
    if (threadIdx.x == 0) s_tile = atomicAdd((unsigned long long*)&hdr->next_tile, 1ull);
    __syncthreads();
    const uint64_t t = wave_uniform(s_tile);  // same tile for the whole workgroup
    __syncthreads();  // every lane has read s_tile before lane 0 overwrites it
    if (t >= total) break;
    batch_tile<U>(d, lg, ts, map, t);
  }
}

// ============================================================== scalar
// One (ctr, key) in the paper's argument order: both generators.
__global__ __launch_bounds__(64) void k_scalar(uint64_t ctr, uint64_t key, uint64_t* out) {
  if (threadIdx.x != 0) return;
  const uint64_t y = ctr * key;
  out[0] = sq32(y, y + key);
  out[1] = sq64(y, y + key);
}

// ============================================================== key-counter mode
// Counter fixed, keys varying (the key-counter usage of Section 4): output j
// comes from keys[j].  Each lane reads 16 / W keys (32 or 16 bytes) and
// writes their outputs as one 16-byte vector, so the kernel streams keys in
// and outputs out at HBM rate; the generator itself is the same as the
// fill's.
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

struct KeysArgs {
  const uint64_t* keys;
  unsigned char* out;
  uint64_t m;
  uint64_t ctr;
  uint64_t nvec;  // full 16-byte output vectors (vector kernel)
};

template <int K>
__device__ __forceinline__ uint64_t keyed_bits(uint64_t ctr, uint64_t key) {
  const uint64_t y = ctr * key;
  return gen_bits<K>(y, y + key);
}

template <int K>
__device__ __forceinline__ void keyed_store(const KeysArgs& a, uint64_t j) {
  const uint64_t v = keyed_bits<K>(a.ctr, a.keys[j]);
  if constexpr (Kind<K>::W == 4) ((uint32_t*)a.out)[j] = (uint32_t)v;
  else ((uint64_t*)a.out)[j] = v;
}

// keys and out 16-byte aligned: vector loads and stores, tail by workgroup 0.
template <int K>
__global__ __launch_bounds__(1024) void k_keys_vec(KeysArgs a) {
  constexpr int E = 16 / Kind<K>::W;
  const u64x2* kp = (const u64x2*)a.keys;
  u32x4* op = (u32x4*)a.out;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll 1
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.nvec; v += stride) {
    u32x4 o;
    if constexpr (E == 4) {
      const u64x2 k0 = kp[2 * v], k1 = kp[2 * v + 1];
      o.x = (uint32_t)keyed_bits<K>(a.ctr, k0.x);
      o.y = (uint32_t)keyed_bits<K>(a.ctr, k0.y);
      o.z = (uint32_t)keyed_bits<K>(a.ctr, k1.x);
      o.w = (uint32_t)keyed_bits<K>(a.ctr, k1.y);
    } else {
      const u64x2 k0 = kp[v];
      const uint64_t b0 = keyed_bits<K>(a.ctr, k0.x), b1 = keyed_bits<K>(a.ctr, k0.y);
      o.x = (uint32_t)b0; o.y = (uint32_t)(b0 >> 32);
      o.z = (uint32_t)b1; o.w = (uint32_t)(b1 >> 32);
    }
    op[v] = o;
  }
  if (blockIdx.x == 0 && threadIdx.x < a.m - a.nvec * E) keyed_store<K>(a, a.nvec * E + threadIdx.x);
}

// Any element-aligned keys/out: one key per lane.
template <int K>
__global__ __launch_bounds__(1024) void k_keys_elem(KeysArgs a) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll 1
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.m; j += stride) keyed_store<K>(a, j);
}

typedef void (*KeysKernel)(KeysArgs);
KeysKernel keys_kernel(int kind, bool vec) {
  switch (kind) {
    case SQ_U32: return vec ? k_keys_vec<0> : k_keys_elem<0>;
    case SQ_F32: return vec ? k_keys_vec<1> : k_keys_elem<1>;
    case SQ_U64: return vec ? k_keys_vec<2> : k_keys_elem<2>;
    default: return vec ? k_keys_vec<3> : k_keys_elem<3>;
  }
}

// ============================================================== key generation
// Distinct-digit keys (Section 3, Discussion: the upper 8 hex digits mutually
// different, the lower 8 too, chosen at random), with an odd least
// significant digit so that ctr -> ctr*key is a bijection mod 2^64.  The
// upper half of key j draws r = squares64(ctr0 + 2j) under gen_key, scales it
// to an index u = floor(r * N / 2^64) over the N = 16!/8! ordered choices of
// 8 digits and reads u's mixed-radix digits (radix 16, 15, ..., 9) as the
// choices of a partial Fisher-Yates shuffle of 0..15.  The lower half draws
// squares64(ctr0 + 2j + 1) and an index over 8 * 15!/8! choices: its radix-8
// digit picks the odd last digit, which is moved to the front of the list,
// and shuffle steps 1..7 take the other seven.  The 16-digit list lives in
// one 64-bit register, one digit per nibble.
constexpr uint64_t kKeyChoicesHi = 518918400ull;  // 16 * 15 * ... * 9
constexpr uint64_t kKeyChoicesLo = 259459200ull;  // 8 * 15 * ... * 9

// Swaps nibbles i and q of the digit list (a no-op when q == i) and returns
// the digit that was at q.
__device__ __forceinline__ uint32_t take_digit(uint64_t& pool, uint32_t i, uint32_t q) {
  const uint64_t dq = (pool >> (4 * q)) & 15, di = (pool >> (4 * i)) & 15;
  pool ^= ((dq ^ di) << (4 * i)) | ((dq ^ di) << (4 * q));
  return (uint32_t)dq;
}

// Shuffle steps 1..7 on the list (step 0 already taken), most significant
// digit first.
__device__ __forceinline__ uint32_t shuffle_digits(uint64_t pool, uint32_t u) {
  uint32_t half = 0;
#pragma unroll
  for (uint32_t i = 1; i < 8; ++i) {
    const uint32_t radix = 16 - i;
    const uint32_t q = i + u % radix;
    u /= radix;
    half = (half << 4) | take_digit(pool, i, q);
  }
  return half;
}

__device__ __forceinline__ uint32_t digits_upper(uint64_t r) {
  uint32_t u = (uint32_t)__umul64hi(r, kKeyChoicesHi);  // < 2^29
  uint64_t pool = 0xFEDCBA9876543210ull;                // nibble p holds digit p
  const uint32_t d0 = take_digit(pool, 0, u % 16);
  u /= 16;
  return (d0 << 28) | shuffle_digits(pool, u);
}

__device__ __forceinline__ uint32_t digits_lower(uint64_t r) {
  uint32_t u = (uint32_t)__umul64hi(r, kKeyChoicesLo);  // < 2^28
  uint64_t pool = 0xFEDCBA9876543210ull;
  const uint32_t odd = take_digit(pool, 0, 2 * (u % 8) + 1);
  u /= 8;
  return (shuffle_digits(pool, u) << 4) | odd;
}

__global__ __launch_bounds__(256) void k_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t* keys) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
#pragma unroll 1
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const uint64_t y = (ctr0 + 2 * j) * gen_key;
    const uint64_t z = y + gen_key, z2 = z + gen_key;
    const uint64_t upper = digits_upper(sq64(y, z)), lower = digits_lower(sq64(z, z2));
    keys[j] = (upper << 32) | lower;
  }
}

}  // namespace

// ============================================================== launchers
namespace sqi {

uint32_t grid_cap(uint32_t block) { return std::min<uint32_t>(0x7FFFFFFFu, 0xFFFFFFFFu / block); }

uint32_t keys_grid(uint64_t work, const sq_launch_cfg& cfg, uint32_t cus) {
  uint64_t grid = (uint64_t)cus * cfg.grid_per_cu;
  const uint64_t need = (work + cfg.block - 1) / cfg.block;
  if (grid > need || cfg.xcd_map == 2) grid = need;  // 2: one step per lane where the grid allows
  grid = std::min<uint64_t>(grid, grid_cap(cfg.block));  // the kernels stride over what is left
  return grid ? (uint32_t)grid : 1;  // the tail still needs a workgroup
}

uint32_t batch_grid(uint64_t tiles_bound, const sq_launch_cfg& cfg, uint32_t cus) {
  const uint64_t grid = cfg.xcd_map == 2 ? tiles_bound : (uint64_t)cus * cfg.grid_per_cu;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(grid, grid_cap(cfg.block)));
}

uint32_t max_segment_chunks(uint32_t block) {
  // one workgroup per chunk: chunk indices and the grid below 2^31, and
  // grid * block below 2^32
  return grid_cap(block);
}

void plan_fill(uint64_t nvec, const sq_launch_cfg& cfg, uint32_t cus, std::vector<FillSegment>& segs) {
  segs.clear();
  const uint64_t per_chunk = (uint64_t)cfg.block * cfg.unroll;
  const uint64_t nchunks = nvec / per_chunk + (nvec % per_chunk != 0);
  // as few launches as the limit allows, with equal shares of the chunks
  const uint64_t maxc = max_segment_chunks(cfg.block);
  const uint64_t nseg = nchunks / maxc + (nchunks % maxc != 0);
  const uint64_t share = nseg > 1 ? nchunks / nseg + (nchunks % nseg != 0) : nchunks;
  uint64_t first = 0;
  do {
    FillSegment g{};
    g.first_chunk = first;
    const uint64_t nc = std::min<uint64_t>(nchunks - first, share);
    const uint64_t vecs = std::min<uint64_t>(nvec - first * per_chunk, nc * per_chunk);
    g.nchunks = (uint32_t)nc;
    g.full = (uint32_t)(vecs / per_chunk);
    g.rem = (uint32_t)(vecs - (uint64_t)g.full * per_chunk);
    g.xcd_map = cfg.xcd_map;
    uint64_t grid = (uint64_t)cus * cfg.grid_per_cu;
    if (grid > nc) grid = nc;
    if (g.xcd_map == 2) {
      grid = nc;  // one chunk per workgroup
    } else if (g.xcd_map == 1 && grid >= 8) {
      grid &= ~7ull;  // XCD-contiguous order needs a multiple of 8
    } else {
      g.xcd_map = 0;
    }
    g.grid = grid ? (uint32_t)grid : 1;  // the head/tail elements still need a workgroup
    segs.push_back(g);
    first += nc;
  } while (first < nchunks);
}

hipError_t launch_fill(int kind, uint64_t key, uint64_t ctr0, uint64_t n, void* out, const sq_launch_cfg& cfg,
                       hipStream_t s, uint64_t step) {
  const int W = kind_bytes(kind), E = 16 / W;
  FillArgs a{};
  a.key = key;
  a.ctr0 = ctr0;
  a.out = (unsigned char*)out;
  // The body starts at a 1 KiB boundary, so each wave's 64 x 16-byte store
  // covers exactly one aligned KiB (whole cache lines, no partial writes).
  const uint32_t mis = (uint32_t)((uintptr_t)out & 1023u);
  uint64_t head = mis ? (1024u - mis) / W : 0;
  if (head > n) head = n;
  a.head = (uint32_t)head;
  const uint64_t nvec = (n - head) / E;
  a.body_nvec = nvec;
  a.tail = (uint32_t)(n - head - nvec * E);
  const bool split = kind == SQ_U32X2 || kind == SQ_F32X2;  // head is even: out is 8-byte aligned
  a.step = step;
  a.dkey = step * key;
  const uint64_t y_body = (ctr0 + (split ? head / 2 : head) * step) * key;
  a.ekey = (uint64_t)(split ? 2 : E) * a.dkey;
  unsigned char* body = a.out + head * W;
  const uint64_t per_chunk = (uint64_t)cfg.block * cfg.unroll;
  std::vector<FillSegment> segs;
  plan_fill(nvec, cfg, (uint32_t)device_info().cus, segs);
  // One chunk of one vector per lane per workgroup: the lane-table kernel,
  // for bodies of at least kLaneMinVec vectors.  Its 2 KiB of arguments cost
  // the host about 0.7 us more per launch, which small fills (whose kernels
  // take microseconds) would feel and large ones do not.
  const bool lanes = cfg.xcd_map == 2 && cfg.unroll == 1 && cfg.block == kLaneBlock && nvec >= kLaneMinVec;
  FillLaneArgs t;
  if (lanes)
    for (uint32_t i = 0; i < kLaneBlock; ++i) t.lane[i] = i * a.ekey;
  const FillKernel k = step == 1 ? fill_kernel<false>(kind, cfg.unroll) : fill_kernel<true>(kind, cfg.unroll);
  const FillLanesKernel kl = step == 1 ? fill_lanes_kernel<false>(kind) : fill_lanes_kernel<true>(kind);
  for (size_t i = 0; i < segs.size(); ++i) {
    const FillSegment& g = segs[i];
    a.body = body + g.first_chunk * per_chunk * 16;
    a.y_body = y_body + g.first_chunk * per_chunk * a.ekey;
    a.nchunks = g.nchunks;
    a.full = g.full;
    a.rem = g.rem;
    a.xcd_map = g.xcd_map;
    a.edges = i == 0;
    if (lanes) {
      t.a = a;
      hipLaunchKernelGGL(kl, dim3(g.grid), dim3(cfg.block), 0, s, t);
    } else {
      hipLaunchKernelGGL(k, dim3(g.grid), dim3(cfg.block), 0, s, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_keys(int kind, uint64_t ctr, const uint64_t* keys, uint64_t m, void* out, const sq_launch_cfg& cfg,
                       hipStream_t s) {
  const int W = kind_bytes(kind), E = 16 / W;
  const bool vec = (((uintptr_t)keys | (uintptr_t)out) & 15) == 0;
  KeysArgs a{keys, (unsigned char*)out, m, ctr, vec ? m / E : 0};
  const uint32_t grid = keys_grid(vec ? a.nvec : m, cfg, (uint32_t)device_info().cus);
  hipLaunchKernelGGL(keys_kernel(kind, vec), dim3(grid), dim3(cfg.block), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_scalar(uint64_t ctr, uint64_t key, uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(64), 0, s, ctr, key, out);
  return hipGetLastError();
}

hipError_t launch_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t* keys, const sq_launch_cfg& cfg,
                            hipStream_t s) {
  const uint32_t B = 256;
  uint64_t grid = (uint64_t)device_info().cus * cfg.grid_per_cu;
  const uint64_t need = (m + B - 1) / B;
  if (grid > need) grid = need;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL(k_make_keys, dim3((uint32_t)grid), dim3(B), 0, s, gen_key, ctr0, m, keys);
  return hipGetLastError();
}

// Workgroups of `k` (with `block` threads) that fit on one CU at once.
static int resident_blocks(const void* k, uint32_t block) {
  static std::mutex mu;
  static std::map<std::pair<const void*, uint32_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({k, block});
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)block, 0) != hipSuccess || nb < 1) nb = 1;
  cache[{k, block}] = nb;
  return nb;
}

hipError_t launch_reduce(int kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out, void* ws,
                         const sq_launch_cfg& cfg, hipStream_t s, uint64_t step) {
  const uint32_t B = 256;  // reduce workgroups are 256 threads (block_sum128 LDS sized for <= 1024)
  const bool queue = cfg.xcd_map == 1;
  ReduceKernel k = step == 1 ? (queue ? reduce_kernel<false, true>(kind, cfg.unroll)
                                      : reduce_kernel<false, false>(kind, cfg.unroll))
                             : (queue ? reduce_kernel<true, true>(kind, cfg.unroll)
                                      : reduce_kernel<true, false>(kind, cfg.unroll));
  const bool split = kind == SQ_U32X2 || kind == SQ_F32X2;
  const uint64_t units = split ? n / 2 : n;  // counters with all their outputs summed
  // Every thread gets the same amount of work, so the grid must be resident
  // at once: a second partial wave of workgroups would double the time.
  const uint32_t gpc = std::min<uint32_t>(cfg.grid_per_cu, (uint32_t)resident_blocks((const void*)k, B));
  uint64_t grid = (uint64_t)device_info().cus * gpc;
  const uint64_t need = (units + B - 1) / B;  // at least one counter per thread
  if (grid > need) grid = need;
  if (grid == 0) grid = 1;
  if (grid > kReduceMaxParts) grid = kReduceMaxParts;
  const uint64_t T = grid * B;
  ReduceArgs a{};
  a.key = key;
  a.ctr0 = ctr0;
  a.n = units;
  a.per = units / T + (units % T != 0);
  a.dkey = step * key;
  a.y0 = ctr0 * key;
  a.partials = (uint64_t*)ws;
  if (queue) {
    // chunks of B * 2^tile_log2 counters, taken from the queue counter that
    // follows the partials in the workspace
    a.per = 1ull << cfg.tile_log2;
    const uint64_t chunk = (uint64_t)B * a.per;
    a.nchunks = units / chunk + (units % chunk != 0);
    if (grid > a.nchunks) grid = a.nchunks ? a.nchunks : 1;
    a.next = (unsigned long long*)((unsigned char*)ws + 16ull * kReduceMaxParts);
    hipLaunchKernelGGL(k_reduce_reset, dim3(1), dim3(64), 0, s, a.next);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  a.ythread = a.per * a.dkey;
  hipLaunchKernelGGL(k, dim3((uint32_t)grid), dim3(B), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int scale = (kind == SQ_F32 || kind == SQ_F32X2) ? -24 : (kind == SQ_F64 ? -53 : 0);
  const int split_tail = (split && (n & 1)) ? kind : 0;
  const uint64_t y_tail = (ctr0 + units * step) * key;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const uint64_t*)ws, (uint32_t)grid, n, scale,
                     split_tail, y_tail, key, out);
  return hipGetLastError();
}

hipError_t launch_reduce_pair(int kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result* out32,
                              sq_sum_result* out64, void* ws, const sq_launch_cfg& cfg, hipStream_t s) {
  const uint32_t B = 256;
  typedef void (*PairKernel)(ReduceArgs, uint64_t*);
  const bool f = kind32 == SQ_F32;
  PairKernel k = cfg.unroll == 1 ? (f ? k_reduce_pair_queue<1, 1> : k_reduce_pair_queue<0, 1>)
               : cfg.unroll == 2 ? (f ? k_reduce_pair_queue<1, 2> : k_reduce_pair_queue<0, 2>)
                                 : (f ? k_reduce_pair_queue<1, 4> : k_reduce_pair_queue<0, 4>);
  const uint32_t gpc = std::min<uint32_t>(cfg.grid_per_cu, (uint32_t)resident_blocks((const void*)k, B));
  uint64_t grid = (uint64_t)device_info().cus * gpc;
  ReduceArgs a{};
  a.key = key;
  a.ctr0 = ctr0;
  a.n = n;
  a.dkey = key;
  a.y0 = ctr0 * key;
  a.per = 1ull << cfg.tile_log2;
  const uint64_t chunk = (uint64_t)B * a.per;
  a.nchunks = n / chunk + (n % chunk != 0);
  if (grid > a.nchunks) grid = a.nchunks ? a.nchunks : 1;
  if (grid > kReduceMaxParts / 2) grid = kReduceMaxParts / 2;  // both partial arrays before the queue counter
  a.ythread = a.per * a.dkey;
  a.partials = (uint64_t*)ws;
  uint64_t* partials64 = (uint64_t*)ws + 2 * grid;
  a.next = (unsigned long long*)((unsigned char*)ws + 16ull * kReduceMaxParts);
  hipLaunchKernelGGL(k_reduce_reset, dim3(1), dim3(64), 0, s, a.next);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3((uint32_t)grid), dim3(B), 0, s, a, partials64);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const uint64_t*)ws, (uint32_t)grid, n, f ? -24 : 0,
                     0, 0ull, key, out32);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, (const uint64_t*)partials64, (uint32_t)grid, n,
                     f ? -53 : 0, 0, 0ull, key, out64);
  return hipGetLastError();
}

// Batch workspace: header, tile_start[m+1] (u64), tile map (u32, one per
// tile).  Tiles are at least 2^10 outputs of at least 4 bytes, and streams
// lie inside the arena without overlap, so there are at most
// m + out_bytes / 2^12 tiles.
uint64_t batch_max_tiles(uint32_t m, uint64_t out_bytes) { return (uint64_t)m + (out_bytes >> 12) + 1; }

size_t batch_ws_bytes(uint32_t m, uint64_t out_bytes) {
  const size_t b = sizeof(BatchHdr) + 8ull * ((size_t)m + 1) + 4ull * batch_max_tiles(m, out_bytes);
  return (b + 255) & ~(size_t)255;
}

hipError_t launch_batch_body(const BatchDesc& d, const uint32_t* m_dev, void* ws, const sq_launch_cfg& cfg,
                             hipStream_t s) {
  BatchHdr* hdr = (BatchHdr*)ws;
  uint64_t* ts = (uint64_t*)((unsigned char*)ws + sizeof(BatchHdr));
  uint32_t* map = (uint32_t*)(ts + (size_t)d.m + 1);
  const uint64_t max_tiles = batch_max_tiles(d.m, d.out_bytes);
  hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(1024), 0, s, d, m_dev, cfg.tile_log2, max_tiles, hdr, ts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_map, dim3(device_info().cus * 4), dim3(256), 0, s, (const BatchHdr*)hdr,
                     (const uint64_t*)ts, map);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // xcd_map 2: one tile per workgroup, grid = the bound on tiles of this
  // size (each stream has at most len / 2^lg + 1 of them, and the streams'
  // outputs of at least 4 bytes fit the arena), capped below 2^32
  // work-items (the kernel strides over tiles past the grid); workgroups
  // past the scanned total exit at once.  Otherwise a persistent grid that
  // takes tiles in a static interleave (0) or from the queue (1).
  const uint64_t tiles_bound = std::min<uint64_t>(max_tiles, (uint64_t)d.m + (d.out_bytes >> (cfg.tile_log2 + 2)) + 1);
  const uint32_t grid = batch_grid(tiles_bound, cfg, (uint32_t)device_info().cus);
  auto k = cfg.unroll == 1 ? k_batch_fill<1> : cfg.unroll == 2 ? k_batch_fill<2>
          : cfg.unroll == 4 ? k_batch_fill<4> : k_batch_fill<8>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(cfg.block), 0, s, d, cfg.tile_log2, cfg.xcd_map, hdr,
                     (const uint64_t*)ts, (const uint32_t*)map);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchDesc& d, void* ws, const sq_launch_cfg& cfg, hipStream_t s) {
  return launch_batch_body(d, nullptr, ws, cfg, s);
}

}  // namespace sqi
