/*
 * squares.h -- C ABI of libsquares.so, the MI355X (gfx950) implementation of
 * the Squares counter-based RNG (B. Widynski, "Squares: A Fast Counter-Based
 * RNG", arXiv 2004.06278).
 *
 * The generators are pure functions of a 64-bit counter and a 64-bit key:
 *   squares32(ctr, key) -> uint32, four rounds          (Section 2)
 *   squares64(ctr, key) -> uint64, five rounds          (Section 5)
 * Each round squares the 64-bit state modulo 2^64, adds ctr*key or
 * (ctr+1)*key (the Weyl terms, Sections 2 and 3) and swaps the two 32-bit
 * halves (Section 3).  The library evaluates them over counter ranges on the
 * GPU; every entry point below launches hand-written HIP kernels and does no
 * generator arithmetic on the host.
 *
 * Conventions shared by every call:
 *  - Pointers named out/ws/keys/... are DEVICE pointers (hipMalloc'd or
 *    torch CUDA tensors) unless stated; the caller owns them and must keep
 *    them valid until the stream work completes.  Nothing on the fill,
 *    reduce and batch paths allocates device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous on that stream; a device fault surfaces at the
 *    next synchronisation, as with any HIP call.
 *  - Counters run ctr0, ctr0+1, ... modulo 2^64: a range that passes
 *    2^64-1 continues at 0 with the same key (the counter is a 64-bit
 *    integer, Section 3).  No error is raised on wrap.
 *  - Any key is accepted, including 0 and even keys; choosing keys with
 *    irregular bit patterns (Section 3) is the caller's concern.
 *  - The argument order of the bulk calls is (key, ctr0); the paper's scalar
 *    functions take (ctr, key).  out[i] == squaresNN(ctr0 + i, key).
 *  - Every call returns an sq_status; sq_last_error() gives a message for
 *    the calling thread's last non-OK status.  No C++ exception crosses the
 *    ABI.
 */
#ifndef SQUARES_H
#define SQUARES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Output kinds.  U32/F32 come from squares32, U64/F64 from squares64.
 * F32 = (squares32 >> 8) * 2^-24 and F64 = (squares64 >> 11) * 2^-53: the
 * paper reports 32-bit and 53-bit precision floating point outputs
 * (Section 5) without a formula; these take the top 24 / 53 bits, which
 * converts exactly into [0, 1).
 * U32X2/F32X2 split each squares64 output into two 32-bit outputs, which
 * Section 5 reports as faster per 32-bit output than squares32: element i
 * comes from counter ctr0 + i/2, the low word for even i and the high word
 * for odd i (the 64-bit output's little-endian order in memory); F32X2
 * converts each word like F32.  Output pointers and batch offsets of the
 * 8-byte kinds and of the split kinds must be 8-byte aligned. */
typedef enum { SQ_U32 = 0, SQ_F32 = 1, SQ_U64 = 2, SQ_F64 = 3, SQ_U32X2 = 4, SQ_F32X2 = 5 } sq_kind;

typedef enum {
    SQ_OK = 0,
    SQ_EINVAL = -1,    /* bad argument (null pointer with n > 0, unknown kind, ...) */
    SQ_EALIGN = -2,    /* pointer or byte offset not a multiple of the element size */
    SQ_ENOMEM = -3,    /* workspace too small, or a request larger than a budget */
    SQ_EHIP = -4,      /* a HIP runtime call failed (message in sq_last_error) */
    SQ_EBUSY = -5,     /* resource in use (e.g. request not finished yet) */
    SQ_ENOTFOUND = -6  /* unknown request id / plan */
} sq_status;

/* Message for the calling thread's most recent non-OK status ("" if none). */
const char *sq_last_error(void);

/* Library version (major*10000 + minor*100 + patch). */
int sq_version(void);

/* Binds the current HIP device, reads its CU count and loads the tuning
 * table from $SQ_TUNE_CACHE if set.  Called implicitly by every entry point;
 * calling it first keeps that work out of a timed region. */
int sq_init(void);

/* ------------------------------------------------------------------------
 * Scalar evaluation in the paper's argument order (ctr, key): squares32
 * (Section 2) and squares64 (Section 5) at one counter, computed by a
 * one-thread kernel on the current device (null stream) and copied back.
 * Synchronous; for spot checks and tests, not for throughput.  `value` is a
 * HOST pointer (null: SQ_EINVAL).  The library keeps one 256-byte device
 * buffer per device for these calls (allocated on first use).
 * ------------------------------------------------------------------------ */
int sq32_at(uint64_t ctr, uint64_t key, uint32_t *value);
int sq64_at(uint64_t ctr, uint64_t key, uint64_t *value);

/* Host helper: the 128-bit integer (hi:lo) times 2^pow2_exp rounded to the
 * nearest double, ties to even -- the rounding sq_reduce applies to its
 * exact sum (scale -24 for F32/F32X2, -53 for F64, 0 for integer kinds). */
double sq_u128_to_double_scaled(uint64_t lo, uint64_t hi, int pow2_exp);

/* ------------------------------------------------------------------------
 * Bulk fills over a counter range (Section 2 squares32, Section 5 squares64).
 *   out[i] = f(ctr0 + i mod 2^64, key),  i in [0, n)
 * `out` must be aligned to 4 bytes (U32, F32) or 8 bytes (other kinds), else
 * SQ_EALIGN; 16-byte alignment is not required (elements up to the first
 * 1 KiB boundary and after the last full 16-byte vector are written one by
 * one).  n == 0 returns SQ_OK without a launch; a
 * null `out` with n > 0 is SQ_EINVAL.  out must hold n elements.  Any n
 * is accepted: a fill whose grid would reach 2^32 work-items is issued as
 * several launches on the same stream.
 * ------------------------------------------------------------------------ */
int sq32_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out, void *stream);
int sq64_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint64_t *out, void *stream);
/* Uniform fills: the conversion is fused into the generating kernel. */
int sq_uniform_f32(uint64_t key, uint64_t ctr0, uint64_t n, float *out, void *stream);
int sq_uniform_f64(uint64_t key, uint64_t ctr0, uint64_t n, double *out, void *stream);
/* The four fills above behind one kind argument. */
int sq_fill(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, void *out, void *stream);
/* The split kinds by name: out[i] = 32-bit word (i & 1) of squares64(ctr0 + i/2). */
int sq64x2_fill(uint64_t key, uint64_t ctr0, uint64_t n, uint32_t *out, void *stream);
int sq_uniform_f32x2(uint64_t key, uint64_t ctr0, uint64_t n, float *out, void *stream);

/* ------------------------------------------------------------------------
 * Launch configurations (chosen by the autotuner; explicit for tests).
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t block;        /* threads per workgroup: 64, 128, 256, 512 or 1024 (fill and
                              batch); the reduce ignores it and always uses 256 */
    uint32_t unroll;       /* 16-byte vectors per lane per chunk: 1, 2, 4 or 8 (fill and
                              batch); outputs per lane per step for reduce: 1, 2 or 4 */
    uint32_t grid_per_cu;  /* workgroups per compute unit (grid = CUs * this), 1..64 */
    uint32_t xcd_map;      /* fill chunk order.  0: grid-stride, consecutive chunks
                              round-robin over the 8 XCDs; 1: grid-stride, each XCD
                              takes one contiguous eighth of the range; 2: one chunk
                              per workgroup (grid = chunks, grid_per_cu unused).
                              reduce: 0 static split over a resident grid; 1 the
                              resident grid takes chunks of 256 * 2^tile_log2
                              counters (tile_log2 6..16) from a queue */
    uint32_t tile_log2;    /* batch: a tile holds 2^tile_log2 * 4 bytes of output
                              (2^tile_log2 outputs of 4-byte kinds, half as many of
                              8-byte kinds), 10..24
                              (batch xcd_map: 0 persistent grid, static interleave;
                              1 persistent grid, tiles taken from a queue in order;
                              2 one tile per workgroup).  reduce with xcd_map 1: the
                              queue's chunk size, as above.  fill: unused */
} sq_launch_cfg;

/* Operation classes the tuning table is keyed by. */
typedef enum { SQ_OP_FILL = 0, SQ_OP_REDUCE = 1, SQ_OP_BATCH = 2 } sq_op;

/* Same as sq_fill with an explicit launch configuration (SQ_EINVAL if the
 * configuration is outside the documented ranges). */
int sq_fill_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, void *out,
                const sq_launch_cfg *cfg, void *stream);

/* Tuning table: one configuration per (op, kind, size bucket), size buckets
 * by n (outputs; for SQ_OP_BATCH the mean stream length):
 * [0,2^16), [2^16,2^20), [2^20,2^24), [2^24,2^28), [2^28,inf). */
int sq_tune_get(sq_op op, sq_kind kind, uint64_t n, sq_launch_cfg *cfg);
int sq_tune_set(sq_op op, sq_kind kind, uint64_t n, const sq_launch_cfg *cfg);
/* Load / save the table as JSON text (host file paths). */
int sq_tune_load(const char *path);
int sq_tune_save(const char *path);
/* Autotuner: for every op/kind it times the candidate configurations on
 * scratch buffers of up to `max_bytes` bytes that it allocates itself (this
 * call is not on the hot path), keeps only candidates whose output is
 * bit-identical to the default configuration's, and stores the fastest in
 * the table.  Fill candidates are timed both right after a compute-bound
 * kernel (a fused sum over 2^31 counters) and back to back, and scored by
 * the sum of the two medians (the shader clock a fill meets depends on what
 * ran before it); reduce and batch candidates back to back.  op_mask bit i
 * selects sq_op i.  Writes the table to `save_path` when non-null.
 * Synchronous. */
int sq_autotune(uint32_t op_mask, uint64_t max_bytes, const char *save_path);

/* ------------------------------------------------------------------------
 * Fused consumer: exact sum over a counter range with no per-element writes.
 * The sum is of the integers whose scaled values are the outputs:
 *   SQ_U32: squares32        SQ_F32: squares32 >> 8   (value = sum * 2^-24)
 *   SQ_U64: squares64        SQ_F64: squares64 >> 11  (value = sum * 2^-53)
 *   SQ_U32X2: each word      SQ_F32X2: each word >> 8 (value = sum * 2^-24)
 * over the same n outputs a fill of that kind would write, as an exact
 * 128-bit integer, so the result does not depend on the order of summation
 * or on the launch configuration.  `value` is that sum times the kind's
 * scale rounded to the nearest double (ties to even).
 * `out` is a DEVICE pointer to one sq_sum_result.  `ws` is a device
 * workspace of at least sq_reduce_workspace_bytes(n) bytes (16-byte
 * aligned), else SQ_ENOMEM: per-workgroup 128-bit partials and the chunk
 * queue counter, which the call resets itself (no caller initialisation;
 * calls that share one workspace must be ordered on one stream).
 * n == 0 writes a zero result.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t lo;     /* low 64 bits of the exact integer sum */
    uint64_t hi;     /* high 64 bits */
    double value;    /* sum * 2^scale rounded to nearest even */
    uint64_t n;      /* number of outputs summed */
} sq_sum_result;

size_t sq_reduce_workspace_bytes(uint64_t n);
int sq_reduce(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result *out,
              void *ws, size_t ws_bytes, void *stream);
int sq_reduce_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result *out,
                  void *ws, size_t ws_bytes, const sq_launch_cfg *cfg, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops): sq_reduce with the workspace
 * taken from a fixed scratch array that the library holds on each device
 * (1 MiB + 256 bytes, in the library's code object, kept until the process
 * ends) instead of a `ws` argument.  Nothing on this path allocates.  The
 * result equals sq_reduce's for the same arguments; `out` is a device
 * pointer to one sq_sum_result (8-byte aligned), n == 0 writes a zero
 * result.  The scratch is shared by every call on a device and keeps the
 * last call's contents: calls that overlap on one device (two streams, two
 * host threads) race and must be ordered on one stream.  Errors: SQ_EINVAL
 * (unknown kind, null out), SQ_EALIGN, SQ_ENOMEM (a workspace need beyond the
 * scratch; sq_reduce_workspace_bytes(n) does not depend on n, so this does
 * not occur for any n today), SQ_EHIP (including a failed lookup of the
 * scratch's device address). */
int sq_reduce_noalloc(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result *out,
                      void *stream);

/* Paired sums: the 32-bit and the 64-bit sum over the same counters in one
 * pass.  squares32 at a counter is the high word of squares64 at it (both
 * compute round 4's t = x*x + z; squares32 returns the high word of t,
 * squares64 keeps t and XORs a value below 2^32 into its low word; Sections
 * 2 and 5), so one squares64 evaluation per counter gives both terms.
 * kind32 = SQ_F32: out32 = sq_reduce(SQ_F32, ...) and out64 =
 * sq_reduce(SQ_F64, ...) over [ctr0, ctr0 + n); kind32 = SQ_U32: the U32 and
 * U64 sums.  Bit-identical to the two separate calls.  `ws` as for
 * sq_reduce (sq_reduce_workspace_bytes(n) bytes, 16-byte aligned); out32
 * and out64 are distinct 8-byte aligned device results.  Errors: SQ_EINVAL
 * (other kinds, null or equal results, invalid cfg: queue order only,
 * xcd_map 1), SQ_EALIGN, SQ_ENOMEM (workspace too small), SQ_EHIP. */
int sq_reduce_pair(sq_kind kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result *out32,
                   sq_sum_result *out64, void *ws, size_t ws_bytes, void *stream);
int sq_reduce_pair_cfg(sq_kind kind32, uint64_t key, uint64_t ctr0, uint64_t n, sq_sum_result *out32,
                       sq_sum_result *out64, void *ws, size_t ws_bytes, const sq_launch_cfg *cfg,
                       void *stream);

/* ------------------------------------------------------------------------
 * Counter increments other than one (Section 4 lists tests of such
 * increments).  Element i is the output of `kind` at counter
 *   ctr0 + i*step (mod 2^64)
 * for U32/F32/U64/F64, and for the split kinds word (i & 1) of squares64 at
 * counter ctr0 + (i/2)*step.  Each counter's second Weyl term stays
 * (ctr+1)*key: the step chooses which counters are visited, the generator
 * is unchanged.  step = 1 gives exactly sq_fill / sq_reduce, step = 0
 * repeats counter ctr0, step = 2^64 - 1 runs the counters backwards.
 * Arguments, alignment, ownership and errors as for sq_fill (fill) and
 * sq_reduce (sum; the sum covers the same n outputs the fill writes).
 * ------------------------------------------------------------------------ */
int sq_fill_strided(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                    void *out, void *stream);
int sq_fill_strided_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                        void *out, const sq_launch_cfg *cfg, void *stream);
int sq_reduce_strided(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                      sq_sum_result *out, void *ws, size_t ws_bytes, void *stream);
int sq_reduce_strided_cfg(sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t step, uint64_t n,
                          sq_sum_result *out, void *ws, size_t ws_bytes,
                          const sq_launch_cfg *cfg, void *stream);

/* ------------------------------------------------------------------------
 * Key-counter mode (Section 4): the counter is fixed and the key varies.
 *   out[j] = f(ctr, keys[j]),  j in [0, m)
 * for kinds U32, F32, U64, F64 (other kinds: SQ_EINVAL).  `keys` is a DEVICE
 * array of m keys (8-byte aligned, else SQ_EALIGN), read once; `out` a device
 * buffer of m elements aligned to the element size.  When both are 16-byte
 * aligned the kernel reads and writes whole 16-byte vectors; otherwise it
 * works one element per lane.  m == 0 returns SQ_OK without a launch.  The
 * _cfg variant takes `block`, `grid_per_cu` and `xcd_map` from cfg
 * (validated as a fill configuration; xcd_map 2 launches one workgroup per
 * block of work instead of a grid-stride loop, as far as a grid below 2^32
 * work-items reaches, and the workgroups stride over the rest; `unroll` and
 * `tile_log2` are ignored).
 * ------------------------------------------------------------------------ */
int sq_fill_keys(sq_kind kind, uint64_t ctr, const uint64_t *keys, uint64_t m, void *out,
                 void *stream);
int sq_fill_keys_cfg(sq_kind kind, uint64_t ctr, const uint64_t *keys, uint64_t m, void *out,
                     const sq_launch_cfg *cfg, void *stream);

/* ------------------------------------------------------------------------
 * Distinct-digit keys on the device (Section 3, Discussion: a key's upper 8
 * hex digits are mutually different, so are its lower 8, and the digits
 * are random); the least significant digit is odd, so ctr -> ctr*key is a
 * bijection mod 2^64.  Key j depends only on (gen_key, ctr0, j):
 *   upper 32 bits: r = squares64(ctr0 + 2j, gen_key), u = floor(r * N / 2^64)
 *   with N = 16*15*...*9 = 518918400, and the digits of a partial
 *   Fisher-Yates shuffle of 0..15 whose step i (i = 0..7) takes the digit at
 *   position i + (u mod (16 - i)) and then sets u = u div (16 - i); the first
 *   digit taken is the most significant.
 *   lower 32 bits: r = squares64(ctr0 + 2j + 1, gen_key),
 *   u = floor(r * 8 * 15*14*...*9 / 2^64); the last digit is the odd digit
 *   2 * (u mod 8) + 1 (then u = u div 8), moved to position 0 of the list;
 *   steps i = 1..7 as above give the other seven digits, most significant
 *   first.
 * (counters mod 2^64).  So windows compose: sq_make_keys(g, c + 2k, ...)
 * yields keys k, k+1, ... of sq_make_keys(g, c, ...).  `keys` is a device
 * array of m uint64 (8-byte aligned, else SQ_EALIGN); m <= 2^62, else
 * SQ_EINVAL.  gen_key should itself be a distinct-digit key.
 * ------------------------------------------------------------------------ */
int sq_make_keys(uint64_t gen_key, uint64_t ctr0, uint64_t m, uint64_t *keys, void *stream);

/* ------------------------------------------------------------------------
 * Ragged batch: m streams in one launch (more keys give more streams,
 * Section 3).  Stream s writes lens[s] outputs of kind kinds[s] from counter
 * ctr0s[s] under keys[s] at byte offset offs[s] of the arena `out` of
 * `out_bytes` bytes.  All five descriptor arrays are DEVICE arrays of m
 * entries; offs[s] must be a multiple of the element size, streams must not
 * overlap (not checked unless $SQ_DEBUG_VALIDATE is set: then the call copies
 * the descriptors to the host, synchronising the stream, and returns
 * SQ_EINVAL / SQ_EALIGN for a stream the kernels would skip or for
 * overlapping ranges).  The kernels check every descriptor on the device:
 * a stream with an unknown kind, a misaligned offset or a range past
 * out_bytes is skipped (nothing written) and counted; sq_batch_errors()
 * reads that count.
 * `ws` needs sq_batch_workspace_bytes(m, out_bytes) bytes (16-byte aligned):
 * a header, the tile scan and a tile-to-stream map sized for the arena.
 * The work is split into tiles of 2^tile_log2 * 4 bytes of output (the
 * configuration's tile_log2); a tile scan, a tile map and one fill kernel
 * run on `stream`.
 * ------------------------------------------------------------------------ */
size_t sq_batch_workspace_bytes(uint32_t m, uint64_t out_bytes);
int sq_fill_batch(const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                  const uint64_t *offs, const uint8_t *kinds, uint32_t m, void *out,
                  uint64_t out_bytes, void *ws, size_t ws_bytes, void *stream);
int sq_fill_batch_cfg(const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                      const uint64_t *offs, const uint8_t *kinds, uint32_t m, void *out,
                      uint64_t out_bytes, void *ws, size_t ws_bytes, const sq_launch_cfg *cfg,
                      void *stream);
/* The same streams as separate launches: one sq_fill kernel per stream,
 * enqueued in order on `stream`.  Here the five descriptor arrays are HOST
 * arrays (checked on the host: SQ_EINVAL / SQ_EALIGN before anything is
 * launched); `out` is the device arena.  This is the per-stream way of
 * producing a batch, kept for comparison with sq_fill_batch. */
int sq_fill_streams(const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                    const uint64_t *offs, const uint8_t *kinds, uint32_t m, void *out,
                    uint64_t out_bytes, void *stream);
/* Number of skipped streams of the last batch that used `ws` (synchronises
 * `stream`). */
int sq_batch_errors(const void *ws, void *stream, uint32_t *count);

/* Batch plan: the tile scan, the tile map and the fill kernel captured once
 * into a HIP graph over fixed descriptor, arena and workspace addresses.  Each
 * launch replays the graph and reads the descriptor arrays' CURRENT
 * contents, so the caller may rewrite keys/ctr0s/lens/offs/kinds (same m)
 * between launches without re-capture. */
typedef struct sq_batch_plan sq_batch_plan;
int sq_batch_plan_create(const uint64_t *keys, const uint64_t *ctr0s, const uint64_t *lens,
                         const uint64_t *offs, const uint8_t *kinds, uint32_t m, void *out,
                         uint64_t out_bytes, void *ws, size_t ws_bytes,
                         const sq_launch_cfg *cfg /* NULL = tuned */, sq_batch_plan **plan);
int sq_batch_plan_launch(sq_batch_plan *plan, void *stream);
int sq_batch_plan_destroy(sq_batch_plan *plan);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching request loop.  The generator is stateless
 * (Section 1, Section 6), so a request's whole state is (key, next counter,
 * outputs left).  Each admitted request's key and counter base (with its
 * kind and output offset) live in a device slot; a tick names each chunk
 * as (slot, first output, count) in a pinned buffer that the tick's first
 * kernel reads, and the kernel derives the chunk's counters from the slot.
 * A request's entries carry its description until one of its ticks has
 * completed, and the tick writes it into the slot, so there are no copies
 * on a control stream and concurrent ticks never wait for each other.
 *  - submit() queues a request; a scheduler thread admits queued requests
 *    in arrival order while free slots and HBM budget allow (the request's
 *    output is carved from a device arena of hbm_budget_bytes owned by the
 *    server), so requests are admitted while others are running.
 *  - Each tick is one run of the batch kernels over the next chunk (at
 *    most chunk_cap outputs) of admitted, unfinished requests, each request
 *    at most once per tick; up to n_streams ticks run concurrently on
 *    separate streams, so consecutive chunks of one request may run at
 *    once on different streams.
 *  - A request's outputs are identical to sq_fill(kind, key, ctr0, n) no
 *    matter what else runs with it.
 *  - Latency = completion seen by the scheduler minus submit() time.
 *  - The scheduler is one host thread per server; while ticks are in flight
 *    it polls their completion events (yielding between polls) for the
 *    lowest latency, so it keeps one host core busy; when idle it sleeps on
 *    a condition variable.
 *  - Errors: if a tick's launch or its completion event reports a HIP
 *    error, the server starts no further tick; submit, poll, wait, result
 *    and latency then return SQ_EHIP (the message names the error), and
 *    destroy frees the server without waiting for the unfinished requests.
 * ------------------------------------------------------------------------ */
typedef struct sq_server sq_server;

typedef struct {
    uint64_t hbm_budget_bytes;  /* output arena size (bytes); every admitted request's
                                   output lives here until released */
    uint32_t max_slots;         /* requests admitted and not yet complete (also the most
                                   chunks in one tick), 1..65536 */
    uint64_t chunk_cap;         /* outputs of one request per tick (>= 4096; rounded down to
                                   an even count so that split-kind chunks start at a low word) */
    uint32_t n_streams;         /* concurrent ticks (one HIP stream each), 1..8.  HIP binds
                                   a stream to one of a few hardware queues (4 per process
                                   by default) when it first runs work; in a process whose
                                   other streams already hold queues, 2 lanes may share one
                                   and serialize, so 4 is the robust choice */
    uint32_t tile_log2;         /* tile of the tick kernel, 10..24 (0 = 14) */
    uint64_t tick_bytes;        /* soft cap on one tick's output bytes (0 = none).  A tick
                                   takes first the requests that finish within one chunk,
                                   then the others round-robin from where the previous tick
                                   stopped, until max_slots entries or this many bytes
                                   (always at least one entry) */
} sq_server_cfg;

/* submit() flags */
#define SQ_SERVE_DISCARD 1u     /* free the output as soon as the request completes */
#define SQ_SERVE_NO_STATS 2u    /* leave this request out of the latency statistics (warm-up) */

typedef struct {
    uint64_t submitted, admitted, completed, released;
    uint64_t outputs, bytes;    /* totals over completed requests */
    uint64_t ticks;
    uint64_t queued_now, active_now, arena_used_bytes;
    double p50_s, p90_s, p99_s, max_s, mean_s;  /* latency over completed requests */
    double first_submit_s, last_complete_s;     /* on the server's steady clock */
} sq_server_stats_t;

int sq_server_create(const sq_server_cfg *cfg, sq_server **srv);
/* SQ_ENOMEM if the request's bytes exceed hbm_budget_bytes (it could never
 * be admitted); SQ_EINVAL for an unknown kind or n == 0. */
int sq_server_submit(sq_server *srv, sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n,
                     uint32_t flags, uint64_t *req_id);
/* *done = 1 once every output of the request is written. */
int sq_server_poll(sq_server *srv, uint64_t req_id, int *done);
/* Blocks until the request completes. */
int sq_server_wait(sq_server *srv, uint64_t req_id);
/* Device address and size of a completed request's output (SQ_EBUSY if not
 * complete; SQ_ENOTFOUND if released or discarded). */
int sq_server_result(sq_server *srv, uint64_t req_id, void **dev_ptr, uint64_t *bytes);
/* Latency of a completed request in seconds. */
int sq_server_latency(sq_server *srv, uint64_t req_id, double *seconds);
/* Returns a completed request's output space to the arena. */
int sq_server_release(sq_server *srv, uint64_t req_id);
/* Cancels a request that is still queued (SQ_EBUSY once admitted). */
int sq_server_cancel(sq_server *srv, uint64_t req_id);
int sq_server_stats(sq_server *srv, sq_server_stats_t *out);
/* Drains admitted work (unless a HIP error stopped the server), then frees the
 * server and its arena; returns SQ_EHIP if the server had failed. */
int sq_server_destroy(sq_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SQUARES_H */
