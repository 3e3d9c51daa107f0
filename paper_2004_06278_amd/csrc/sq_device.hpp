// Device primitives of the Squares generators for gfx950.
//
// A round of either generator (Section 2 for squares32, Section 5 for
// squares64) is
//     x <- x*x + a (mod 2^64);  x <- x rotated by 32 bits
// with a the first Weyl term y = ctr*key in odd rounds and the second one
// z = (ctr+1)*key in even rounds.  On CDNA the 64-bit state lives in two
// 32-bit VGPRs (xl, xh) and
//     x*x mod 2^64 = xl*xl + ((2*xl*xh) mod 2^32) * 2^32,
// so a round is one v_mad_u64_u32 (xl*xl + a, full 64-bit result), one
// v_mul_lo_u32 (xl*xh) and one v_lshl_add_u32 (the doubled cross term added
// into the high word).  The rotation is free: it only swaps which register
// is called "low".  No MFMA: nothing here is a contraction.
//
// Consecutive counters share Weyl terms: z(c) = y(c+1), and y advances by
// key per counter (Section 2: ctr*key replaces the sequence w += s), so a
// lane that owns counters c..c+E-1 needs E+1 values y(c)..y(c+E), each one
// 64-bit add from the previous.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sqd {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Returns v unchanged, but opaque to the optimizer; the empty asm emits no
// instruction.  Used on per-chunk base values so that loop-strength
// reduction does not turn each unrolled vector's Weyl term and address into
// an induction variable of its own.
__device__ __forceinline__ uint64_t opaque(uint64_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// The same for a workgroup-uniform value, kept in scalar registers: stops
// LLVM from folding a uniform term back into a per-lane product.
__device__ __forceinline__ uint64_t opaque_uniform(uint64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// A value every lane of the wave holds (e.g. broadcast through LDS), moved
// to scalar registers so the code that depends on it stays scalar.
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// yc + tid*ekey (mod 2^64) for a wave-uniform yc and ekey: the first Weyl
// term of the vector lane `tid` owns when consecutive lanes own consecutive
// vectors.  The high word of tid*ekey's upper part is added to yc first
// (one 32-bit multiply and add), then one 32x32->64 multiply-add supplies
// tid times the low word of ekey with its carry.  Written out because LLVM
// otherwise builds the 64-bit product with an extra multiply-add and
// register moves, which this per-lane setup cannot afford where a lane
// computes only one 16-byte vector.
__device__ __forceinline__ uint64_t lane_weyl(uint64_t yc, uint64_t ekey, uint32_t tid) {
  const uint32_t hi = (uint32_t)(yc >> 32) + tid * (uint32_t)(ekey >> 32);
  const uint64_t a = ((uint64_t)hi << 32) | (uint32_t)yc;
  uint64_t t;
  asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=&v"(t) : "v"(tid), "s"((uint32_t)ekey), "v"(a) : "vcc");
  return t;
}

// The two instruction groups of a round, each pinned with a non-volatile
// asm statement so that LLVM can schedule them but not rewrite them (with
// plain C it duplicates the multiply-add, strength-reduces round 1's y*y + y
// into a polynomial in the loop counter, or turns the cross term into a
// three-instruction shift/move/multiply-add form).
//   m  = xl*xl + a                 one v_mad_u64_u32 (carry-out to vcc, unread;
//                                  early-clobber: dst must not overlap srcs)
//   hi = m_hi + 2*xl*xh mod 2^32   v_mul_lo_u32 + v_lshl_add_u32
__device__ __forceinline__ uint64_t sq_lo_plus(uint32_t xl, uint64_t a) {
  uint64_t m;
  asm("v_mad_u64_u32 %0, vcc, %1, %1, %2" : "=&v"(m) : "v"(xl), "v"(a) : "vcc");
  return m;
}

__device__ __forceinline__ uint32_t cross_add(uint32_t xl, uint32_t xh, uint32_t m_hi) {
  uint32_t hi;
  asm("v_mul_lo_u32 %0, %1, %2\n\tv_lshl_add_u32 %0, %0, 1, %3" : "=&v"(hi) : "v"(xl), "v"(xh), "v"(m_hi));
  return hi;
}

// rot32(x*x + a)
__device__ __forceinline__ uint64_t round_rot(uint64_t x, uint64_t a) {
  const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
  const uint64_t m = sq_lo_plus(xl, a);
  const uint32_t hi = cross_add(xl, xh, (uint32_t)(m >> 32));
  return ((uint64_t)(uint32_t)m << 32) | hi;  // halves swapped: no instruction
}

// x*x + a without the rotation, as (lo, hi) words
__device__ __forceinline__ void round_norot(uint64_t x, uint64_t a, uint32_t& lo, uint32_t& hi) {
  const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
  const uint64_t m = sq_lo_plus(xl, a);
  lo = (uint32_t)m;
  hi = cross_add(xl, xh, (uint32_t)(m >> 32));
}

// Upper 32 bits of x*x + a
__device__ __forceinline__ uint32_t round_hi(uint64_t x, uint64_t a) {
  const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
  const uint64_t m = sq_lo_plus(xl, a);
  return cross_add(xl, xh, (uint32_t)(m >> 32));
}

// x*x + a (mod 2^64), not rotated.  Round 1 of both generators is
// rot32(y*y + y): its value before the rotation, r1 = y*y + y, is what the
// functions below take when a caller supplies it from a running difference
// (see fd_step) instead of squaring.
__device__ __forceinline__ uint64_t square_plus(uint64_t x, uint64_t a) {
  uint32_t lo, hi;
  round_norot(x, a, lo, hi);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t rot32(uint64_t v) { return (v << 32) | (v >> 32); }  // a register swap

// squares32 from round 1's value r1 = y*y + y and the Weyl terms y = ctr*key,
// z = (ctr+1)*key.
__device__ __forceinline__ uint32_t sq32_after1(uint64_t r1, uint64_t y, uint64_t z) {
  uint64_t x = rot32(r1);        // round 1's rotation
  x = round_rot(x, z);           // round 2
  x = round_rot(x, y);           // round 3
  return round_hi(x, z);         // round 4: upper half of x*x + z
}

__device__ __forceinline__ uint32_t sq32(uint64_t y, uint64_t z) { return sq32_after1(square_plus(y, y), y, z); }

// squares64 from round 1's value: round 4 keeps t = x*x + z whole; round 5
// squares rot32(t), adds y and its upper 32 bits are XORed into the low word
// of t.
__device__ __forceinline__ uint64_t sq64_after1(uint64_t r1, uint64_t y, uint64_t z) {
  uint64_t x = rot32(r1);
  x = round_rot(x, z);
  x = round_rot(x, y);
  uint32_t tl, th;
  round_norot(x, z, tl, th);                          // t = (th:tl)
  const uint64_t xr = ((uint64_t)tl << 32) | th;      // rot32(t)
  const uint32_t r5 = round_hi(xr, y);
  return ((uint64_t)th << 32) | (tl ^ r5);
}

__device__ __forceinline__ uint64_t sq64(uint64_t y, uint64_t z) { return sq64_after1(square_plus(y, y), y, z); }

// Round 1 by running differences.  Along Weyl terms y, y+s, y+2s, ...
// (s = key for consecutive counters, s = step*key for counters `step` apart,
// s = J*key for counters J apart) round 1's value r1(y) = y*y + y is a
// quadratic in the position, so modulo 2^64
//     r1(y + s) = r1(y) + d(y),   d(y) = 2*s*y + s*s + s,
//     d(y + s)  = d(y) + 2*s*s,
// two 64-bit adds per counter instead of one squaring (three instructions).
// The state is (r1, d) at the current y; s2 = 2*s, c = s*s + s and
// dd = 2*s*s are the step's uniform constants.
struct FdConst {
  uint64_t s2, c, dd;
};
__device__ __forceinline__ FdConst fd_const(uint64_t s) {
  FdConst k;
  k.s2 = 2 * s;
  k.c = s * s + s;
  k.dd = 2 * s * s;
  return k;
}
// d at y: 2*s*y + s*s + s
__device__ __forceinline__ uint64_t fd_diff(uint64_t y, const FdConst& k) { return y * k.s2 + k.c; }

// Exact conversions to [0,1): top 24 bits of a squares32 output, top 53 bits
// of a squares64 output, each scaled by a power of two.
__device__ __forceinline__ float to_f32(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }
// (u >> 11) * 2^-53 in five exact steps: the high word and the low word with
// its low 11 bits cleared convert exactly, hi * 2^32 + lo has at most 53
// significant bits (so the fused multiply-add is exact), and scaling by
// 2^-64 is exact (the result is 0 or at least 2^-53).
__device__ __forceinline__ double to_f64(uint64_t u) {
  const double hi = (double)(uint32_t)(u >> 32);
  const double lo = (double)((uint32_t)u & 0xFFFFF800u);
  return __builtin_fma(hi, 0x1p32, lo) * 0x1p-64;
}

// Output-kind traits.  Kind numbering matches sq_kind in squares.h.
//   W:     bytes per output element
//   CPV:   counters consumed by one 16-byte vector of outputs
//   SPLIT: each squares64 output gives two 32-bit elements (low word first)
template <int K> struct Kind;
template <> struct Kind<0> { static constexpr int W = 4, CPV = 4; static constexpr bool SPLIT = false; };  // U32
template <> struct Kind<1> { static constexpr int W = 4, CPV = 4; static constexpr bool SPLIT = false; };  // F32
template <> struct Kind<2> { static constexpr int W = 8, CPV = 2; static constexpr bool SPLIT = false; };  // U64
template <> struct Kind<3> { static constexpr int W = 8, CPV = 2; static constexpr bool SPLIT = false; };  // F64
template <> struct Kind<4> { static constexpr int W = 4, CPV = 2; static constexpr bool SPLIT = true; };   // U32X2
template <> struct Kind<5> { static constexpr int W = 4, CPV = 2; static constexpr bool SPLIT = true; };   // F32X2

// One output of non-split kind K for the counter whose Weyl terms are
// (y, z), as raw bits (low word first for 8-byte kinds).
template <int K>
__device__ __forceinline__ uint64_t gen_bits(uint64_t y, uint64_t z) {
  if constexpr (K == 0) return sq32(y, z);
  if constexpr (K == 1) return __float_as_uint(to_f32(sq32(y, z)));
  if constexpr (K == 2) return sq64(y, z);
  if constexpr (K == 3) return (uint64_t)__double_as_longlong(to_f64(sq64(y, z)));
}

// Both 32-bit elements of a split kind from one squares64 output.
template <int K>
__device__ __forceinline__ void split_pair(uint64_t y, uint64_t z, uint32_t& lo, uint32_t& hi) {
  const uint64_t v = sq64(y, z);
  lo = (uint32_t)v;
  hi = (uint32_t)(v >> 32);
  if constexpr (K == 5) {
    lo = __float_as_uint(to_f32(lo));
    hi = __float_as_uint(to_f32(hi));
  }
}

// Sixteen bytes of consecutive outputs starting at the counter with first
// Weyl term y0: four 32-bit outputs (squares32, or two split squares64
// outputs) or two 64-bit outputs.
template <int K>
__device__ __forceinline__ u32x4 gen_vec(uint64_t y0, uint64_t key) {
  u32x4 o;
  if constexpr (Kind<K>::SPLIT) {
    const uint64_t y1 = y0 + key, y2 = y1 + key;
    uint32_t a, b, c, d;
    split_pair<K>(y0, y1, a, b);
    split_pair<K>(y1, y2, c, d);
    o.x = a; o.y = b; o.z = c; o.w = d;
  } else if constexpr (Kind<K>::W == 4) {
    const uint64_t y1 = y0 + key, y2 = y1 + key, y3 = y2 + key, y4 = y3 + key;
    o.x = (uint32_t)gen_bits<K>(y0, y1);
    o.y = (uint32_t)gen_bits<K>(y1, y2);
    o.z = (uint32_t)gen_bits<K>(y2, y3);
    o.w = (uint32_t)gen_bits<K>(y3, y4);
  } else {
    const uint64_t y1 = y0 + key, y2 = y1 + key;
    const uint64_t a = gen_bits<K>(y0, y1), b = gen_bits<K>(y1, y2);
    o.x = (uint32_t)a; o.y = (uint32_t)(a >> 32);
    o.z = (uint32_t)b; o.w = (uint32_t)(b >> 32);
  }
  return o;
}

// The same sixteen bytes when consecutive outputs are `step` counters apart
// (Section 4 tests increments other than one): the first Weyl terms advance
// by dkey = step*key, and each output's second term is its own first term
// plus key, since z(c) = (c+1)*key no longer equals y of the next output.
template <int K>
__device__ __forceinline__ u32x4 gen_vec_strided(uint64_t y0, uint64_t key, uint64_t dkey) {
  u32x4 o;
  if constexpr (Kind<K>::SPLIT) {
    const uint64_t y1 = y0 + dkey;
    uint32_t a, b, c, d;
    split_pair<K>(y0, y0 + key, a, b);
    split_pair<K>(y1, y1 + key, c, d);
    o.x = a; o.y = b; o.z = c; o.w = d;
  } else if constexpr (Kind<K>::W == 4) {
    const uint64_t y1 = y0 + dkey, y2 = y1 + dkey, y3 = y2 + dkey;
    o.x = (uint32_t)gen_bits<K>(y0, y0 + key);
    o.y = (uint32_t)gen_bits<K>(y1, y1 + key);
    o.z = (uint32_t)gen_bits<K>(y2, y2 + key);
    o.w = (uint32_t)gen_bits<K>(y3, y3 + key);
  } else {
    const uint64_t y1 = y0 + dkey;
    const uint64_t a = gen_bits<K>(y0, y0 + key), b = gen_bits<K>(y1, y1 + key);
    o.x = (uint32_t)a; o.y = (uint32_t)(a >> 32);
    o.z = (uint32_t)b; o.w = (uint32_t)(b >> 32);
  }
  return o;
}

// Counter offset of element i of a range (split kinds: two elements per
// counter).
template <int K>
__device__ __forceinline__ uint64_t elem_ctr(uint64_t i) {
  return Kind<K>::SPLIT ? i >> 1 : i;
}

// Writes element i of a range that starts at counter ctr0 and visits every
// step-th counter (element store, for heads and tails); p is the element's
// address.
template <int K>
__device__ __forceinline__ void store_elem(unsigned char* p, uint64_t ctr0, uint64_t i, uint64_t key,
                                           uint64_t step = 1) {
  const uint64_t y = (ctr0 + elem_ctr<K>(i) * step) * key;
  if constexpr (Kind<K>::SPLIT) {
    uint32_t lo, hi;
    split_pair<K>(y, y + key, lo, hi);
    *(uint32_t*)p = (i & 1) ? hi : lo;
  } else {
    const uint64_t v = gen_bits<K>(y, y + key);
    if constexpr (Kind<K>::W == 4) *(uint32_t*)p = (uint32_t)v;
    else *(uint64_t*)p = v;
  }
}

// The integer a reduce of kind K sums for one counter (the value is that
// integer times 2^-24 for F32 and F32X2 and 2^-53 for F64), from round 1's
// value r1 and the Weyl terms.  Split kinds sum both halves of the
// counter's squares64 output.
template <int K>
__device__ __forceinline__ uint64_t sum_term_after1(uint64_t r1, uint64_t y, uint64_t z) {
  if constexpr (K == 0) return sq32_after1(r1, y, z);
  if constexpr (K == 1) return sq32_after1(r1, y, z) >> 8;
  if constexpr (K == 2) return sq64_after1(r1, y, z);
  if constexpr (K == 3) return sq64_after1(r1, y, z) >> 11;
  if constexpr (K == 4) {
    const uint64_t v = sq64_after1(r1, y, z);
    return (v & 0xFFFFFFFFull) + (v >> 32);
  }
  if constexpr (K == 5) {
    const uint64_t v = sq64_after1(r1, y, z);
    return (((uint32_t)v) >> 8) + (v >> 40);
  }
}

// The low-half term of a split kind (the last element of an odd count).
template <int K>
__device__ __forceinline__ uint64_t split_lo_term(uint64_t y, uint64_t z) {
  const uint32_t lo = (uint32_t)sq64(y, z);
  return K == 5 ? (lo >> 8) : lo;
}

}  // namespace sqd
