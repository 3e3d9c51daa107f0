// Continuous-batching request server.
//
// The generators are stateless (a request is fully described by kind, key,
// starting counter and length), so an admitted request's key and counter
// state is one 32-byte device slot: key, first counter, output offset, kind.
// A tick names each chunk as (slot, first output, count) and its first
// kernel derives the chunk's counter and output address from the slot.  The
// slot is written by the request's own ticks: until a tick holding the
// request has completed, its entries carry the whole description, which the
// tick stores in the slot (identical values from any lane), so there are no
// copies on a control stream and ticks on different lanes never wait for
// each other; chunks of one request may run on several lanes at once.
//
// A scheduler thread loops:
//   1. retire ticks whose completion event has fired; a request completes
//      when all of its outputs were scheduled and no tick holding one of its
//      chunks is still running;
//   2. admit queued requests in arrival order while a slot is free and the
//      output arena (hbm_budget_bytes, owned by the server) has room;
//   3. if a tick stream is idle and some admitted request has outputs left,
//      build a tick: the next chunk (at most chunk_cap outputs) of such
//      requests, written into that stream's pinned tick buffer, which the
//      tick's first kernel reads directly; then (with the lock released)
//      launch the tick's four kernels on the stream (expand -> tile scan ->
//      tile map -> persistent fill).  Direct launches: on MI355X they gave
//      a lower open-loop latency than replaying a captured graph of the
//      same kernels (p50 0.098 against 0.110 ms at half capacity).
// Up to n_streams ticks are in flight at once, so requests admitted while
// others run share the device with them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "sq_internal.hpp"

using namespace sqi;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

enum class St { Queued, Active, Done };

struct Req {
  uint64_t id;
  int kind;
  uint64_t key, ctr0, n;
  uint32_t flags;
  St st = St::Queued;
  uint64_t off = 0, bytes = 0;  // arena range
  uint32_t slot = 0;            // device slot holding the key and counter state
  bool slot_ready = false;      // a tick holding this request has completed (the slot is written)
  uint64_t next = 0;            // next output to schedule
  uint32_t inflight = 0;        // running ticks that hold a chunk of this request
  double t_submit = 0, t_done = 0;
};

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = (bytes + 255) & ~255ull;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = (bytes + 255) & ~255ull;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0;
};

// ---------------------------------------------------------------- slots and ticks
// An admitted request's key and counter base live in a device slot for the
// request's lifetime; each tick names a chunk as (slot, first,
// count).  Until a tick holding the request has completed, its entries also
// carry the whole description (init = 1), which the tick writes into the
// slot (every such write stores the same values).
struct SlotDev {
  uint64_t key;
  uint64_t ctr0;       // counter of the request's first output
  uint64_t out_off;    // arena byte offset of the request's output
  uint32_t kind;
  uint32_t pad;
};
static_assert(sizeof(SlotDev) == 32, "slot is 32 bytes");
struct TickEntry {
  uint32_t slot;
  uint32_t init;
  uint64_t first;      // first output of the chunk within the request (even for split kinds)
  uint64_t count;      // outputs in this chunk
  uint64_t key;        // init only
  uint64_t ctr0;       // init only
  uint64_t out_off;    // init only
  uint32_t kind;       // init only
  uint32_t pad;
};
static_assert(sizeof(TickEntry) == 56, "tick entry is 56 bytes");
struct TickHdr {
  uint32_t entries;    // number of TickEntry that follow
  uint32_t pad;
  uint64_t pad2[7];
};
static_assert(sizeof(TickHdr) == 64, "tick header is 64 bytes");

// ---------------------------------------------------------------- tick expansion
// Turns the tick's chunk entries into batch descriptors: a chunk's key,
// first counter and output offset come from its request's device slot
// (written first from the entry while the entry carries the description).
__global__ __launch_bounds__(256) void k_tick_expand(const TickHdr* th, const TickEntry* ent,
                                                     SlotDev* slots, uint64_t* keys, uint64_t* ctr0s,
                                                     uint64_t* lens, uint64_t* offs, uint8_t* kinds,
                                                     uint32_t* m_out, uint32_t max_entries) {
  const uint32_t m = th->entries < max_entries ? th->entries : max_entries;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *m_out = m;
  if (i >= m) return;
  const TickEntry e = ent[i];
  SlotDev s;
  if (e.init) {
    s.key = e.key;
    s.ctr0 = e.ctr0;
    s.out_off = e.out_off;
    s.kind = e.kind;
    s.pad = 0;
    slots[e.slot] = s;
  } else {
    s = slots[e.slot];
  }
  const uint32_t W = (s.kind == 2 || s.kind == 3) ? 8u : 4u;
  keys[i] = s.key;
  ctr0s[i] = s.ctr0 + (s.kind > 3 ? e.first >> 1 : e.first);  // split kinds: two outputs per counter
  lens[i] = e.count;
  offs[i] = s.out_off + e.first * W;
  kinds[i] = (uint8_t)s.kind;
}

// tick ws layout: keys, ctr0s, lens, offs (u64 x max each), kinds (u8 x max,
// padded), m (u32, padded to 256), then the batch workspace over the arena.
size_t tick_ws_bytes(uint32_t max_entries, uint64_t arena_bytes) {
  const size_t arrays = 32ull * max_entries + (((size_t)max_entries + 255) & ~(size_t)255) + 256;
  return arrays + batch_ws_bytes(max_entries, arena_bytes);
}

hipError_t launch_tick(const void* tick_buf, SlotDev* slots, uint32_t max_entries, unsigned char* arena,
                       uint64_t arena_bytes, void* tick_ws, const sq_launch_cfg& cfg, hipStream_t s) {
  unsigned char* w = (unsigned char*)tick_ws;
  uint64_t* keys = (uint64_t*)w;
  uint64_t* ctr0s = keys + max_entries;
  uint64_t* lens = ctr0s + max_entries;
  uint64_t* offs = lens + max_entries;
  uint8_t* kinds = (uint8_t*)(offs + max_entries);
  uint32_t* m_dev = (uint32_t*)(kinds + (((size_t)max_entries + 255) & ~(size_t)255));
  void* bws = (unsigned char*)m_dev + 256;
  const TickHdr* th = (const TickHdr*)tick_buf;
  const TickEntry* ent = (const TickEntry*)((const unsigned char*)tick_buf + sizeof(TickHdr));
  const uint32_t blocks = (max_entries + 255) / 256;
  hipLaunchKernelGGL(k_tick_expand, dim3(blocks), dim3(256), 0, s, th, ent, slots, keys, ctr0s, lens, offs, kinds,
                     m_dev, max_entries);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchDesc d{keys, ctr0s, lens, offs, kinds, max_entries, arena, arena_bytes};
  return launch_batch_body(d, m_dev, bws, cfg, s);
}

struct TickLane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  unsigned char* host_buf = nullptr;  // pinned: TickHdr + entries, read by the device
  void* ws = nullptr;                 // device tick workspace
  bool busy = false;                  // a tick was built for this lane and has not retired
  bool finished = false;              // its completion event fired (scheduler thread only)
  hipError_t status = hipSuccess;     // event status at completion
  std::vector<uint64_t> reqs;         // requests with a chunk in the running tick
};

}  // namespace

struct sq_server {
  sq_server_cfg cfg{};
  sq_launch_cfg lcfg{};
  int device = 0;
  unsigned char* arena_dev = nullptr;
  SlotDev* slots_dev = nullptr;       // max_slots request descriptions, written by the ticks
  std::vector<TickLane> lanes;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  std::vector<uint64_t> active;       // admitted, not complete, in admission order
  size_t rr = 0;                      // round-robin start in `active` for ticks under a byte cap
  std::vector<uint32_t> free_slots;
  std::unordered_set<uint64_t> cancelled;
  Arena* arena = nullptr;
  uint64_t next_id = 1;
  bool stop = false;
  std::string fatal;                  // first HIP error seen by the scheduler
  std::thread th;

  std::vector<double> lat;            // latencies of completed requests
  uint64_t submitted = 0, admitted = 0, completed = 0, released = 0, outputs = 0, bytes_done = 0, ticks = 0;
  double first_submit = 0, last_complete = 0;

  void loop();
  bool retire_locked();
  bool admit_locked();
  bool build_tick_locked(TickLane* L);
  void finish_locked(Req& r);
};

void sq_server::finish_locked(Req& r) {
  r.st = St::Done;
  r.t_done = now_s();
  if (!(r.flags & SQ_SERVE_NO_STATS)) lat.push_back(r.t_done - r.t_submit);
  ++completed;
  outputs += r.n;
  bytes_done += r.bytes;
  last_complete = r.t_done;
  free_slots.push_back(r.slot);
  active.erase(std::find(active.begin(), active.end(), r.id));
  if (r.flags & SQ_SERVE_DISCARD) {
    arena->release(r.off, r.bytes);
    ++released;
    const uint64_t id = r.id;  // r dies with the erase
    reqs.erase(id);
  }
  cv_done.notify_all();
}

// Retires the lanes whose tick finished (their `finished` flag was set by
// the scheduler outside the lock); returns true if any retired.
bool sq_server::retire_locked() {
  bool any = false;
  for (auto& L : lanes) {
    if (!L.finished) continue;
    if (L.status != hipSuccess && fatal.empty()) fatal = std::string("tick: ") + hipGetErrorString(L.status);
    L.finished = false;
    L.busy = false;
    any = true;
    for (uint64_t id : L.reqs) {
      Req& r = reqs.at(id);
      r.slot_ready = true;
      if (--r.inflight == 0 && r.next == r.n) finish_locked(r);
    }
    L.reqs.clear();
  }
  return any;
}

// Admits queued requests (FIFO) while fewer than max_slots are active and
// the arena has room.
bool sq_server::admit_locked() {
  bool any = false;
  while (!queue.empty() && !free_slots.empty()) {
    Req& r = reqs.at(queue.front());
    uint64_t off = 0;
    if (!arena->alloc(r.bytes, &off)) break;  // head of line waits for room
    queue.pop_front();
    r.off = off;
    r.slot = free_slots.back();
    free_slots.pop_back();
    r.st = St::Active;
    active.push_back(r.id);
    ++admitted;
    any = true;
  }
  return any;
}

// Fills idle lane L's pinned tick buffer with the next chunk of admitted
// requests that have outputs left; returns false (L stays idle) if there
// are none.  The launch itself happens outside the lock.
bool sq_server::build_tick_locked(TickLane* L) {
  TickHdr* th_ = (TickHdr*)L->host_buf;
  TickEntry* ent = (TickEntry*)(L->host_buf + sizeof(TickHdr));
  uint32_t m = 0;
  uint64_t bytes = 0;
  const uint64_t cap = cfg.tick_bytes ? cfg.tick_bytes : UINT64_MAX;
  auto add = [&](Req& r) {
    const uint64_t cnt = std::min<uint64_t>(cfg.chunk_cap, r.n - r.next);
    const uint32_t W = (uint32_t)kind_bytes(r.kind);
    TickEntry& te = ent[m];
    te = TickEntry{};
    te.slot = r.slot;
    te.first = r.next;
    te.count = cnt;
    if (!r.slot_ready) {  // the slot may not be written yet: carry the description
      te.init = 1;
      te.key = r.key;
      te.ctr0 = r.ctr0;
      te.out_off = r.off;
      te.kind = (uint32_t)r.kind;
    }
    r.next += cnt;
    ++r.inflight;
    L->reqs.push_back(r.id);
    bytes += cnt * W;
    ++m;
  };
  // requests that finish within this chunk first (they leave the tick done),
  // then the others from the round-robin position while under the byte cap
  auto mine = [](const Req& r) { return r.next < r.n; };
  for (uint64_t id : active) {
    if (m == cfg.max_slots) break;
    Req& r = reqs.at(id);
    if (mine(r) && r.n - r.next <= cfg.chunk_cap) add(r);
  }
  // each request at most once per tick: one pass over `active` from a fixed
  // start (a slot must not appear twice in a tick)
  const size_t na = active.size(), start = rr;
  for (size_t k = 0; k < na && m < cfg.max_slots && (bytes < cap || m == 0); ++k) {
    const size_t i = (start + k) % na;
    Req& r = reqs.at(active[i]);
    if (!mine(r)) continue;
    add(r);
    rr = i + 1;
  }
  if (m == 0) return false;
  th_->entries = m;
  L->busy = true;
  ++ticks;
  return true;
}

// The scheduler.  Lane state (busy, finished, event status) belongs to this
// thread; request, queue and arena state is shared and changed only
// under `mu`.  HIP calls (event queries, kernel launches) run
// with the lock released, so submit()/poll() never wait behind them.
void sq_server::loop() {
  // the launch helpers size their grids from this thread's device binding;
  // without the server's device no tick may start
  const hipError_t de = hipSetDevice(device);
  if (de != hipSuccess || ensure_init() != SQ_OK) {
    std::lock_guard<std::mutex> g(mu);
    fatal = std::string("scheduler thread cannot bind device ") + std::to_string(device) +
            (de != hipSuccess ? std::string(": ") + hipGetErrorString(de) : std::string());
  }
  std::vector<TickLane*> to_launch;
  for (;;) {
    for (auto& L : lanes) {
      if (!L.busy || L.finished) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipErrorNotReady) continue;
      L.status = q;
      L.finished = true;
    }
    bool progress = false, inflight = false, exit_now = false;
    to_launch.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      progress |= retire_locked();
      progress |= admit_locked();
      // after a HIP error no further tick starts: the admitted requests stay
      // incomplete and every call reports the error
      for (auto& L : lanes)
        if (fatal.empty() && !L.busy && build_tick_locked(&L)) to_launch.push_back(&L);
      inflight = std::any_of(lanes.begin(), lanes.end(), [](const TickLane& l) { return l.busy; });
      if (stop && !inflight && ((active.empty() && queue.empty()) || !fatal.empty())) exit_now = true;
      else if (!inflight && !progress) cv_work.wait_for(lk, std::chrono::milliseconds(20));
    }
    if (exit_now) break;
    hipError_t e = hipSuccess;
    std::atomic_thread_fence(std::memory_order_seq_cst);  // tick entries visible before the launch doorbell
    for (TickLane* L : to_launch) {
      if (e == hipSuccess)
        e = launch_tick(L->host_buf, slots_dev, cfg.max_slots, arena_dev, cfg.hbm_budget_bytes, L->ws, lcfg, L->stream);
      if (e == hipSuccess) e = hipEventRecord(L->done, L->stream);
      if (e != hipSuccess) {  // the lane never runs: retire it at once with the error
        L->status = e;
        L->finished = true;
      }
    }
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> g(mu);
      if (fatal.empty()) fatal = std::string("server launch: ") + hipGetErrorString(e);
    }
    if (!progress && to_launch.empty() && inflight) std::this_thread::yield();  // ticks running: poll again
  }
}

static void server_free(sq_server* s) {
  for (auto& L : s->lanes) {
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.host_buf) (void)hipHostFree(L.host_buf);
    if (L.ws) (void)hipFree(L.ws);
  }
  if (s->slots_dev) (void)hipFree(s->slots_dev);
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  delete s->arena;
  delete s;
}

extern "C" {

int sq_server_create(const sq_server_cfg* cfg, sq_server** out) {
  if (cfg == nullptr || out == nullptr) return fail(SQ_EINVAL, "null cfg or server pointer");
  *out = nullptr;
  if (cfg->hbm_budget_bytes < 4096 || cfg->max_slots < 1 || cfg->max_slots > 65536 || cfg->chunk_cap < 4096 ||
      cfg->n_streams < 1 || cfg->n_streams > 8 || (cfg->tile_log2 != 0 && (cfg->tile_log2 < 10 || cfg->tile_log2 > 24)))
    return fail(SQ_EINVAL, "server configuration out of range");
  int rc = ensure_init();
  if (rc != SQ_OK) return rc;
  sq_server* s = new sq_server();
  s->cfg = *cfg;
  s->cfg.chunk_cap &= ~1ull;  // chunks of split kinds must start at a low word
  s->device = device_info().device;
  // Ticks are many small batches over a large arena: a persistent grid with
  // the static tile interleave (no tile-bound grid, no queue) and 2^14-output
  // tiles gave the lowest latency in open-loop runs on MI355X.
  s->lcfg = sq_launch_cfg{256, 8, 4, 0, 14};
  if (cfg->tile_log2) s->lcfg.tile_log2 = cfg->tile_log2;
  s->arena = new Arena(cfg->hbm_budget_bytes);
  hipError_t e = hipMalloc((void**)&s->arena_dev, cfg->hbm_budget_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&s->slots_dev, sizeof(SlotDev) * cfg->max_slots);
  s->lanes.resize(cfg->n_streams);
  const size_t tbuf = sizeof(TickHdr) + sizeof(TickEntry) * (size_t)cfg->max_slots;
  for (auto& L : s->lanes) {
    if (e != hipSuccess) break;
    e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&L.host_buf, tbuf, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&L.ws, tick_ws_bytes(cfg->max_slots, cfg->hbm_budget_bytes));
    if (e != hipSuccess) break;
    ((TickHdr*)L.host_buf)->entries = 0;
  }
  if (e != hipSuccess) {
    int r = fail_hip(e, "server setup");
    server_free(s);
    return r;
  }
  for (uint32_t i = 0; i < cfg->max_slots; ++i) s->free_slots.push_back(cfg->max_slots - 1 - i);
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return SQ_OK;
}

int sq_server_submit(sq_server* s, sq_kind kind, uint64_t key, uint64_t ctr0, uint64_t n, uint32_t flags,
                     uint64_t* req_id) {
  if (s == nullptr || req_id == nullptr) return fail(SQ_EINVAL, "null server or id pointer");
  const int W = kind_bytes(kind);
  if (W == 0) return fail(SQ_EINVAL, "unknown kind " + std::to_string((int)kind));
  if (n == 0) return fail(SQ_EINVAL, "empty request");
  if (n > s->cfg.hbm_budget_bytes / W || ((n * W + 255) & ~255ull) > s->cfg.hbm_budget_bytes)
    return fail(SQ_ENOMEM, "request larger than the server's HBM budget");
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->fatal.empty()) return fail(SQ_EHIP, "server failed: " + s->fatal);
  if (s->stop) return fail(SQ_EBUSY, "server is shutting down");
  Req r;
  r.id = s->next_id++;
  r.kind = kind;
  r.key = key;
  r.ctr0 = ctr0;
  r.n = n;
  r.flags = flags;
  r.bytes = n * W;
  r.t_submit = now_s();
  if (s->submitted == 0) s->first_submit = r.t_submit;
  ++s->submitted;
  s->reqs.emplace(r.id, r);
  s->queue.push_back(r.id);
  *req_id = r.id;
  s->cv_work.notify_one();
  return SQ_OK;
}

int sq_server_poll(sq_server* s, uint64_t id, int* done) {
  if (s == nullptr || done == nullptr) return fail(SQ_EINVAL, "null server or flag pointer");
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->fatal.empty()) return fail(SQ_EHIP, "server failed: " + s->fatal);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    if (id == 0 || id >= s->next_id || s->cancelled.count(id)) return fail(SQ_ENOTFOUND, "unknown or cancelled request");
    *done = 1;  // completed and already released or discarded
    return SQ_OK;
  }
  *done = it->second.st == St::Done;
  return SQ_OK;
}

int sq_server_wait(sq_server* s, uint64_t id) {
  if (s == nullptr) return fail(SQ_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (id == 0 || id >= s->next_id || s->cancelled.count(id)) return fail(SQ_ENOTFOUND, "unknown or cancelled request");
  for (;;) {
    if (!s->fatal.empty()) return fail(SQ_EHIP, "server failed: " + s->fatal);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second.st == St::Done) return SQ_OK;
    s->cv_done.wait_for(lk, std::chrono::milliseconds(50));
  }
}

int sq_server_result(sq_server* s, uint64_t id, void** ptr, uint64_t* bytes) {
  if (s == nullptr || ptr == nullptr || bytes == nullptr) return fail(SQ_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->fatal.empty()) return fail(SQ_EHIP, "server failed: " + s->fatal);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(SQ_ENOTFOUND, "unknown, released or discarded request");
  if (it->second.st != St::Done) return fail(SQ_EBUSY, "request not complete");
  *ptr = s->arena_dev + it->second.off;
  *bytes = it->second.bytes;
  return SQ_OK;
}

int sq_server_latency(sq_server* s, uint64_t id, double* seconds) {
  if (s == nullptr || seconds == nullptr) return fail(SQ_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  if (!s->fatal.empty()) return fail(SQ_EHIP, "server failed: " + s->fatal);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(SQ_ENOTFOUND, "unknown, released or discarded request");
  if (it->second.st != St::Done) return fail(SQ_EBUSY, "request not complete");
  *seconds = it->second.t_done - it->second.t_submit;
  return SQ_OK;
}

int sq_server_release(sq_server* s, uint64_t id) {
  if (s == nullptr) return fail(SQ_EINVAL, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(SQ_ENOTFOUND, "unknown or already released request");
  if (it->second.st != St::Done) return fail(SQ_EBUSY, "request not complete");
  s->arena->release(it->second.off, it->second.bytes);
  ++s->released;
  s->reqs.erase(it);
  s->cv_work.notify_one();
  return SQ_OK;
}

int sq_server_cancel(sq_server* s, uint64_t id) {
  if (s == nullptr) return fail(SQ_EINVAL, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(SQ_ENOTFOUND, "unknown request");
  if (it->second.st != St::Queued) return fail(SQ_EBUSY, "request already admitted");
  s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
  s->reqs.erase(it);
  s->cancelled.insert(id);
  return SQ_OK;
}

int sq_server_stats(sq_server* s, sq_server_stats_t* o) {
  if (s == nullptr || o == nullptr) return fail(SQ_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *o = sq_server_stats_t{};
  o->submitted = s->submitted;
  o->admitted = s->admitted;
  o->completed = s->completed;
  o->released = s->released;
  o->outputs = s->outputs;
  o->bytes = s->bytes_done;
  o->ticks = s->ticks;
  o->queued_now = s->queue.size();
  o->active_now = s->active.size();
  o->arena_used_bytes = s->arena->used();
  o->first_submit_s = s->first_submit;
  o->last_complete_s = s->last_complete;
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto q = [&](double p) { return v[std::min<size_t>(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
    o->p50_s = q(0.50);
    o->p90_s = q(0.90);
    o->p99_s = q(0.99);
    o->max_s = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    o->mean_s = sum / (double)v.size();
  }
  return SQ_OK;
}

int sq_server_destroy(sq_server* s) {
  if (s == nullptr) return SQ_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    // queued requests never start; admitted ones drain
    for (uint64_t id : s->queue) {
      s->reqs.erase(id);
      s->cancelled.insert(id);
    }
    s->queue.clear();
    s->stop = true;
    s->cv_work.notify_all();
  }
  s->th.join();
  std::string fatal = s->fatal;
  // the scheduler exits only with no tick in flight; synchronizing the lane
  // streams (not the device) leaves the caller's other work alone
  hipError_t e = hipSuccess;
  for (auto& L : s->lanes) {
    const hipError_t le = hipStreamSynchronize(L.stream);
    if (e == hipSuccess) e = le;
  }
  server_free(s);
  if (!fatal.empty()) return fail(SQ_EHIP, "server failed: " + fatal);
  if (e != hipSuccess) return fail_hip(e, "server drain");
  return SQ_OK;
}

}  // extern "C"
