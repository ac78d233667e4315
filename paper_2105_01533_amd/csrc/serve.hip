// Continuous-batching server over the batched tick (see include/sparsesim.h,
// srv_*).
//
// Requests (a circuit and a state configuration) queue in FIFO order and are
// admitted while their device footprint fits the pool and a slot is free.
// Each tick takes one segment from every running request -- a fused
// phase/permutation run, one branching gate, or one measurement, exactly as
// the single-state engine would cut it, a run together with the gate right
// after it -- uploads one work list, replays the
// captured tick graph, and reads back every slot's control words.  Finished
// requests are copied to host memory and their device memory is returned to
// the pool, which lets queued requests in on the next tick.
//
// Requests of large capacity take the large-state lane instead: host threads
// run each through the single-state engine (sim_apply_gates on a workspace
// from the pool, on a stream per thread), whole, while the ticks go on.  A
// tick is as long as its longest item, and a large state's runs would hold
// every small request in the tick for as long; on the lane a large request
// also needs no host round trip per gate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/sparsesim.h"
#include "host_pool.h"
#include "run_compiler.h"
#include "sim_internal.h"

using namespace sparsesim;

namespace {

thread_local std::string g_srv_error;

int sfail(int code, const std::string& msg) {
  g_srv_error = msg;
  return code;
}

#define SRV_HIP(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return sfail(SIM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kA = 256;
constexpr uint64_t kMinArena = 1ull << 20;   // smallest per-tick op arena
size_t al(size_t x) { return (x + kA - 1) / kA * kA; }

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint64_t index_slots(uint64_t n, double lf) {
  const uint64_t want = (uint64_t)std::ceil((double)(n ? n : 1) / lf) + 1;
  return std::max<uint64_t>(64, pow2_at_least(want));
}

double lf_or_default(double lf) { return lf > 0.0 ? lf : 0.5; }

// First-fit allocator over [0, size) with coalescing (offsets 256-aligned).
struct Pool {
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
    used = peak = 0;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    used -= n;
    auto it = free_.emplace(off, n).first;
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
};

struct Footprint {
  size_t lo[2], hi[2], amp[2], table, partner, tot, cnt1, part, total;
  uint64_t slots, units;
};

Footprint footprint_of(const sim_config& c, double lf) {
  Footprint f{};
  const uint64_t cap = c.capacity;
  const bool wide = c.n_qubits > 64;
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    f.lo[b] = off;
    off += al(cap * 8);
    f.hi[b] = off;
    if (wide) off += al(cap * 8);
    f.amp[b] = off;
    off += al(cap * 16);
  }
  f.slots = index_slots(cap, lf);
  f.table = off;
  off += al(f.slots * 8);
  f.partner = off;
  off += al(cap * 4);
  f.units = (cap + kChunk - 1) / kChunk + 1;
  f.tot = off;
  off += al(f.units * 4);
  f.cnt1 = off;
  off += al(f.units * 4);
  f.part = off;
  off += al(f.units * 16);
  f.total = off;
  return f;
}

enum SegKind { SEG_NONE = 0, SEG_MONO, SEG_U2, SEG_MEAS };

// Allocator whose resize leaves new elements uninitialised (they are written
// whole right after).
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};

struct Request {
  uint64_t id = 0;
  sim_config cfg{};
  sim_key basis{};
  std::vector<sim_gate, NoInit<sim_gate>> gates;
  std::vector<size_t> mono_op;        // MONO ordinal -> op index
  RunCompiler rc;
  bool compiled = false;              // descriptors and bit-sliced ops built (at admission)
  int32_t state = SRV_QUEUED;
  int32_t error = SIM_OK;
  // device placement
  Footprint fp{};
  size_t off = 0;
  int slot = -1;
  Buf buf[2]{};
  uint64_t* table = nullptr;
  uint32_t *partner = nullptr, *tot = nullptr, *cnt1 = nullptr;
  double2* part = nullptr;
  int cur = 0;
  uint64_t nnz = 1;
  // progress
  size_t i = 0;
  size_t mono_seen = 0;
  bool deferred = false;              // its last fused run did not fit the tick's arena
  bool copied = false;                // final state copied to the result arrays
  hipError_t copy_err = hipSuccess;
  // A background host job (compile, grouping or copy out) is in flight for
  // this request; what it writes is the tick thread's to read once this is
  // false (stored under the server's bg_mu, read with acquire).
  std::atomic<bool> bg_busy{false};
  // Grouping of the fused run expected next, made while the previous tick ran
  // on the GPU; used only if the run that comes is exactly [b, b + len).
  struct Ahead {
    bool valid = false;
    size_t b = 0, len = 0;
    bool rp = false;                  // a register-plane program (prog), else groups (grp)
    BsRun br{};
    std::vector<BsGroup> grp;
    std::vector<RpRec> prog;
  } ahead;
  bool large = false;                 // runs on the large-state lane
  int lane_rc = SIM_OK;               // the lane's result code
  SegKind seg = SEG_NONE;
  // Measurements this tick: the first and the ones right after it, which run
  // in later launch rounds of the same tick (op indices).
  uint32_t chain_len = 0;
  size_t chain_op[kMaxChain] = {};
  sim_stats st{};
  std::vector<int32_t> outcomes;
  // result (storage order; res_hi only for more than 64 qubits)
  uint64_t res_n = 0;
  std::unique_ptr<uint64_t[]> res_lo, res_hi;
  std::unique_ptr<sim_c64[]> res_amp;

  // Result arrays for n entries (left uninitialised: they are written whole).
  void alloc_result(uint64_t n) {
    res_n = n;
    res_lo.reset(new uint64_t[std::max<uint64_t>(n, 1)]);
    res_hi.reset(cfg.n_qubits > 64 ? new uint64_t[std::max<uint64_t>(n, 1)] : nullptr);
    res_amp.reset(new sim_c64[std::max<uint64_t>(n, 1)]);
  }
};

}  // namespace

struct srv_t {
  srv_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* pool_mem = nullptr;
  bool own_pool = false;
  Pool pool;
  SlotCtl* d_ctl = nullptr;
  Ctl* d_rpctl = nullptr;             // counters of the register-plane launches (not reported)
  SlotCtl* h_ctl = nullptr;
  std::vector<int> free_slots;
  // tick buffer (same layout host/device): header | items | units | ops arena
  char* d_tick = nullptr;
  char* h_tick = nullptr;
  size_t items_off = 0, units_off = 0, arena_off = 0, tick_bytes = 0;
  size_t max_items = 0, max_units = 0;   // capacity of the item and unit areas
  size_t chain_hdr_off = 0;               // headers of a tick's later measurement rounds
  // One captured graph per non-empty set of kernel families (index = family
  // mask), so a tick replays only the kernels it has items for.
  hipGraph_t graph[16] = {};
  hipGraphExec_t exec[16] = {};
  int grid = 2048;
  uint32_t run_ops = 4096;            // longest fused run per request per tick (ops)
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<uint64_t> queue;
  std::vector<Request*> running;
  srv_stats stats{};
  int device = 0;
  // large-state lane
  uint64_t lane_cap = 0;              // capacity from which a request takes the lane (0: no lane)
  std::deque<uint64_t> lane_queue;    // queued large requests (FIFO)
  int lane_in_flight = 0;             // admitted to the lane, not yet folded back (tick thread)
  std::vector<std::thread> lane_threads;
  std::vector<hipStream_t> lane_streams;
  int lane_depth = 0;                 // lane requests admitted at once (workers + 1)
  std::mutex lane_mu;
  std::condition_variable lane_cv, lane_done_cv;
  std::deque<Request*> lane_todo;     // admitted, waiting for the lane thread
  std::vector<Request*> lane_done;    // finished by the lane thread
  bool lane_stop = false;
  double lane_ms = 0.0;               // lane thread only (read under lane_mu)
  // Background host workers (host work only; a copy out reads device memory
  // with hipMemcpy): compiling submitted circuits, grouping the runs requests
  // are expected to take next, copying finished states out.
  std::vector<std::thread> bg_threads;
  std::mutex bg_mu;
  std::condition_variable bg_cv, bg_done_cv;
  std::deque<std::pair<Request*, int>> bg_urgent, bg_normal;   // groupings; compiles and copies
  bool bg_stop = false;
  double bg_copy_ms = 0.0;            // under bg_mu
  std::vector<Request*> copying;      // finished, state being copied out (tick thread)
};

namespace {

int capture_tick(srv_t* s) {
  const auto* hdr = reinterpret_cast<const BTick*>(s->d_tick);
  const auto* items = reinterpret_cast<const BItem*>(s->d_tick + s->items_off);
  const auto* units = reinterpret_cast<const uint32_t*>(s->d_tick + s->units_off);
  if (s->cfg.flags & SRV_FLAG_NO_GRAPH) return SIM_OK;
  for (uint32_t m = 1; m <= kFamAll; ++m) {
    SRV_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    launch_batch_tick(s->stream, hdr, items, units, s->grid, m);
    hipGraph_t g = nullptr;
    SRV_HIP(hipStreamEndCapture(s->stream, &g));
    s->graph[m] = g;
    SRV_HIP(hipGraphInstantiate(&s->exec[m], s->graph[m], nullptr, nullptr, 0));
  }
  return SIM_OK;
}

// Longest fused run whose ops always fit an empty arena (bit-sliced groups or
// per-entry descriptors, worst case): a run is cut there whatever else shares
// the tick, so a request's runs -- and with them its rounding -- are the same
// alone and in any mix.  A MONO op compiles to at most three bit-sliced ops;
// the rewrite of uncontrolled X gates at most doubles them and adds one per
// qubit; a group holds at least one op; a register-plane program has at most
// rp_records_bound records.
uint64_t arena_run_cap(const srv_t* s, const Request& r) {
  const uint64_t groups = s->cfg.arena_bytes / sizeof(BsGroup);
  const uint64_t by_groups = groups > r.cfg.n_qubits ? (groups - r.cfg.n_qubits) / (2 * 3) : 1;
  const uint64_t by_desc = s->cfg.arena_bytes / sizeof(MonoDesc);
  // A register-plane program of L ops has at most rp_records_bound(3 L, nq)
  // records: 8 (6 L + nq) + 16.
  const uint64_t recs = s->cfg.arena_bytes / sizeof(RpRec);
  const uint64_t fixed = 8ull * r.cfg.n_qubits + 16;
  const uint64_t by_prog = recs > fixed ? (recs - fixed) / 48 : 1;
  return std::max<uint64_t>(1, std::min({by_groups, by_desc, by_prog}));
}

// Bit-sliced fused runs of states of at least this many entries take the
// register-plane kernel, one launch per run on the server's stream ahead of
// the tick's graph (two waves per SIMD on 2048-entry tiles, about twice the
// LDS-plane tile's speed on large states; the two give the same bits).
constexpr uint64_t kRpMinEntries = 1ull << 16;

bool use_rp(const srv_t* s, uint64_t nnz) {
  return !(s->cfg.flags & SRV_FLAG_NO_RP) && nnz >= kRpMinEntries;
}

// Position in a request's op list.
struct Cursor {
  size_t i, mono_seen;
  uint64_t skipped;   // branching gates skipped by the cap
};

// The segment that starts at c for a state of nnz entries; advances c past it.
// Reads only the request's ops and configuration.
SegKind scan_segment(const srv_t* s, const Request& r, uint64_t nnz, Cursor& c, size_t* begin, size_t* len,
                     size_t* op) {
  uint64_t fuse_max = std::min<uint64_t>(r.cfg.fuse_max ? r.cfg.fuse_max : 65536u, s->run_ops);
  if (s->cfg.tick_updates) fuse_max = std::min<uint64_t>(fuse_max, std::max<uint64_t>(1, s->cfg.tick_updates / std::max<uint64_t>(nnz, 1)));
  fuse_max = std::min<uint64_t>(fuse_max, arena_run_cap(s, r));
  size_t run_len = 0, run_begin = c.mono_seen;
  const size_t n = r.gates.size();
  while (c.i < n) {
    const sim_gate& g = r.gates[c.i];
    if (g.op == SIM_OP_MONO) {
      if (!run_len) run_begin = c.mono_seen;
      ++run_len;
      ++c.mono_seen;
      ++c.i;
      if (run_len >= fuse_max) break;
      continue;
    }
    if (g.op == SIM_OP_U2 && g.cap && 2 * nnz > g.cap) {
      ++c.skipped;
      ++c.i;
      continue;
    }
    if (run_len) break;
    *op = c.i++;
    return g.op == SIM_OP_U2 ? SEG_U2 : SEG_MEAS;
  }
  if (run_len) {
    *begin = run_begin;
    *len = run_len;
    return SEG_MONO;
  }
  return SEG_NONE;
}

// Next segment of r, consuming skipped branching gates; sets r.seg and the
// run [begin, begin + len) of MONO ordinals or the op index of the gate.
SegKind next_segment(srv_t* s, Request& r, size_t* begin, size_t* len, size_t* op) {
  Cursor c{r.i, r.mono_seen, 0};
  const SegKind k = scan_segment(s, r, r.nnz, c, begin, len, op);
  r.i = c.i;
  r.mono_seen = c.mono_seen;
  r.st.u2_skipped += c.skipped;
  return k;
}

// The request's final state into its host result.  Touches only r, so it
// may run for several requests at once on the host thread pool.
hipError_t copy_out(Request& r) {
  r.alloc_result(r.nnz);
  const Buf& b = r.buf[r.cur];
  const bool wide = r.cfg.n_qubits > 64;
  const hipError_t e = copy_state_to_host_soa(b.key_lo, wide ? b.key_hi : nullptr, b.amp, r.nnz, r.res_lo.get(),
                                              wide ? r.res_hi.get() : nullptr, r.res_amp.get());
  if (e == hipSuccess) r.copied = true;
  return e;
}

int finish(srv_t* s, Request& r, int32_t state, int32_t err) {
  r.state = state;
  r.error = err;
  if (state == SRV_DONE) {
    if (!r.copied) SRV_HIP(copy_out(r));
    r.st.gates_applied = r.gates.size();
    s->stats.completed++;
  } else {
    s->stats.failed++;
  }
  r.st.peak_nnz = std::max<uint64_t>(r.st.peak_nnz, r.nnz);
  s->pool.release(r.off, r.fp.total);
  s->free_slots.push_back(r.slot);
  r.slot = -1;
  r.gates.clear();
  r.gates.shrink_to_fit();
  r.rc = RunCompiler{};
  r.ahead = Request::Ahead{};
  return SIM_OK;
}

// Descriptors and bit-sliced ops of a request's circuit.
void compile_request(Request& r) {
  for (size_t i = 0; i < r.gates.size(); ++i)
    if (r.gates[i].op == SIM_OP_MONO) {
      r.rc.descs.push_back(mono_desc(r.gates[i]));
      r.mono_op.push_back(i);
    }
  r.rc.pair_window = 64;   // grouping happens on the tick's critical path
  if (r.cfg.mono_mode != SIM_MONO_DIRECT) r.rc.compile(r.cfg.n_qubits);
  else r.rc.n_qubits = r.cfg.n_qubits;
  r.compiled = true;
}

// ---- large-state lane ----------------------------------------------------------
// One request, whole, through the single-state engine on the lane's stream;
// the state is copied out to the request's host result.  Runs on the lane
// thread; touches only the request (the tick thread does not, meanwhile).
void lane_run(srv_t* s, Request& r, hipStream_t stream) {
  sim_t* h = nullptr;
  size_t n_meas = 0;
  for (const sim_gate& g : r.gates) n_meas += g.op == SIM_OP_MEASURE;
  std::vector<int32_t> outs(n_meas);
  int rc = sim_create(&r.cfg, stream, s->pool_mem + r.off, r.fp.total, &h);
  if (rc == SIM_OK) rc = sim_set_basis(h, r.basis);
  if (rc == SIM_OK) rc = sim_apply_gates(h, r.gates.data(), r.gates.size(), outs.data(), &r.st);
  uint64_t n = 0;
  if (rc == SIM_OK) rc = sim_nnz(h, &n);
  if (rc == SIM_OK) {
    r.alloc_result(n);
    uint64_t got = 0;
    rc = sim_export_state_soa(h, r.res_lo.get(), r.res_hi.get(), r.res_amp.get(), n, &got);
  }
  if (h) (void)sim_destroy(h);
  r.outcomes.assign(outs.begin(), outs.begin() + std::min<size_t>(outs.size(), r.st.measures));
  r.lane_rc = rc;
}

void lane_main(srv_t* s, hipStream_t stream) {
  (void)hipSetDevice(s->device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->lane_mu);
      s->lane_cv.wait(lk, [&] { return s->lane_stop || !s->lane_todo.empty(); });
      if (s->lane_todo.empty()) return;   // stopping
      r = s->lane_todo.front();
      s->lane_todo.pop_front();
    }
    const auto t0 = std::chrono::steady_clock::now();
    lane_run(s, *r, stream);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    {
      std::lock_guard<std::mutex> lk(s->lane_mu);
      s->lane_ms += ms;
      s->lane_done.push_back(r);
    }
    s->lane_done_cv.notify_all();
  }
}

// Fold the lane's finished requests back (tick thread): result state, pool
// memory, counters.
void lane_fold(srv_t* s) {
  std::vector<Request*> fin;
  {
    std::lock_guard<std::mutex> lk(s->lane_mu);
    fin.swap(s->lane_done);
    s->stats.lane_ms = s->lane_ms;
  }
  for (Request* r : fin) {
    --s->lane_in_flight;
    s->pool.release(r->off, r->fp.total);
    r->state = r->lane_rc == SIM_OK ? SRV_DONE : SRV_FAILED;
    r->error = r->lane_rc;
    if (r->state == SRV_DONE) s->stats.completed++;
    else s->stats.failed++;
    s->stats.lane_completed++;
    r->gates.clear();
    r->gates.shrink_to_fit();
  }
}

// Admit large requests in FIFO order while the pool has room: one per lane
// worker and one more waiting with its memory, so no worker idles between
// requests.
void lane_admit(srv_t* s) {
  while (!s->lane_queue.empty() && s->lane_in_flight < s->lane_depth) {
    Request& r = *s->reqs[s->lane_queue.front()];
    size_t off;
    if (!s->pool.alloc(r.fp.total, &off)) break;
    s->lane_queue.pop_front();
    r.off = off;
    r.state = SRV_RUNNING;
    ++s->lane_in_flight;
    s->stats.admitted++;
    {
      std::lock_guard<std::mutex> lk(s->lane_mu);
      s->lane_todo.push_back(&r);
    }
    s->lane_cv.notify_one();
  }
}

// ---- background host workers -------------------------------------------------
enum BgKind { BG_COMPILE, BG_GROUP, BG_COPY };
constexpr int kBgThreads = 8;

double bg_ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Queue a job for r (at most one in flight per request).  A grouping job
// finds its run in r.ahead (b, len, br), set by the caller beforehand.
void bg_push(srv_t* s, Request* r, BgKind k) {
  r->bg_busy.store(true, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(s->bg_mu);
    (k == BG_GROUP ? s->bg_urgent : s->bg_normal).emplace_back(r, (int)k);
  }
  s->bg_cv.notify_one();
}

void bg_main(srv_t* s) {
  (void)hipSetDevice(s->device);
  HostPool::run_serially_here();
  for (;;) {
    std::pair<Request*, int> job;
    {
      std::unique_lock<std::mutex> lk(s->bg_mu);
      s->bg_cv.wait(lk, [&] { return s->bg_stop || !s->bg_urgent.empty() || !s->bg_normal.empty(); });
      if (s->bg_stop) return;
      auto& q = s->bg_urgent.empty() ? s->bg_normal : s->bg_urgent;
      job = q.front();
      q.pop_front();
    }
    Request& r = *job.first;
    double ms = 0.0;
    switch (job.second) {
      case BG_COMPILE:
        compile_request(r);
        break;
      case BG_GROUP:
        if (r.ahead.rp) r.rc.schedule(r.ahead.b, r.ahead.len, r.ahead.prog, &r.ahead.br);
        else r.rc.group(r.ahead.b, r.ahead.len, r.ahead.grp, &r.ahead.br);
        r.ahead.valid = true;
        break;
      case BG_COPY: {
        const auto t0 = std::chrono::steady_clock::now();
        r.copy_err = copy_out(r);
        ms = bg_ms_since(t0);
        break;
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->bg_mu);
      s->bg_copy_ms += ms;
      r.bg_busy.store(false, std::memory_order_release);
    }
    s->bg_done_cv.notify_all();
  }
}

// Wait until r has no background job in flight.
void bg_wait(srv_t* s, Request* r) {
  std::unique_lock<std::mutex> lk(s->bg_mu);
  s->bg_done_cv.wait(lk, [&] { return !r->bg_busy.load(std::memory_order_acquire); });
}

// Wait (at most `us` microseconds) for any background job to finish.
void bg_wait_any(srv_t* s, int us) {
  std::unique_lock<std::mutex> lk(s->bg_mu);
  s->bg_done_cv.wait_for(lk, std::chrono::microseconds(us));
}

void bg_shutdown(srv_t* s) {
  {
    std::lock_guard<std::mutex> lk(s->bg_mu);
    s->bg_stop = true;
    s->bg_urgent.clear();   // jobs running now finish; queued ones are dropped
    s->bg_normal.clear();
  }
  s->bg_cv.notify_all();
  for (auto& t : s->bg_threads) t.join();
  s->bg_threads.clear();
}

// Admission uploads read from these (and from the request and the pinned
// control words), which outlive the copies.
const double kUnitAmp[2] = {1.0, 0.0};

// Admits queued requests in FIFO order while memory and slots last.  Their
// circuits are compiled in the background from submission on; a request
// takes no segment until that is done.
int admit(srv_t* s) {
  lane_admit(s);
  while (!s->queue.empty() && !s->free_slots.empty()) {
    Request& r = *s->reqs[s->queue.front()];
    size_t off;
    if (!s->pool.alloc(r.fp.total, &off)) break;        // FIFO: wait for memory
    s->queue.pop_front();
    r.off = off;
    r.slot = s->free_slots.back();
    s->free_slots.pop_back();
    char* base = s->pool_mem + off;
    const bool wide = r.cfg.n_qubits > 64;
    for (int b = 0; b < 2; ++b) {
      r.buf[b].key_lo = reinterpret_cast<uint64_t*>(base + r.fp.lo[b]);
      r.buf[b].key_hi = wide ? reinterpret_cast<uint64_t*>(base + r.fp.hi[b]) : nullptr;
      r.buf[b].amp = reinterpret_cast<double2*>(base + r.fp.amp[b]);
    }
    r.table = reinterpret_cast<uint64_t*>(base + r.fp.table);
    r.partner = reinterpret_cast<uint32_t*>(base + r.fp.partner);
    r.tot = reinterpret_cast<uint32_t*>(base + r.fp.tot);
    r.cnt1 = reinterpret_cast<uint32_t*>(base + r.fp.cnt1);
    r.part = reinterpret_cast<double2*>(base + r.fp.part);
    r.cur = 0;
    r.nnz = 1;
    // initial basis state and control words
    SlotCtl c{};
    c.nnz[0] = 1;
    c.outcome = -1;
    s->h_ctl[r.slot] = c;
    SRV_HIP(hipMemcpyAsync(&s->d_ctl[r.slot], &s->h_ctl[r.slot], sizeof(SlotCtl), hipMemcpyHostToDevice,
                           s->stream));
    SRV_HIP(hipMemcpyAsync(r.buf[0].key_lo, &r.basis.lo, 8, hipMemcpyHostToDevice, s->stream));
    if (wide) SRV_HIP(hipMemcpyAsync(r.buf[0].key_hi, &r.basis.hi, 8, hipMemcpyHostToDevice, s->stream));
    SRV_HIP(hipMemcpyAsync(r.buf[0].amp, kUnitAmp, 16, hipMemcpyHostToDevice, s->stream));
    r.state = SRV_RUNNING;
    s->running.push_back(&r);
    s->stats.admitted++;
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

size_t srv_footprint(const sim_config* cfg) {
  if (!cfg || cfg->n_qubits < 1 || cfg->n_qubits > 128 || cfg->capacity < 1 || cfg->capacity >= (1ull << 31))
    return 0;
  return footprint_of(*cfg, lf_or_default(cfg->load_factor)).total;
}

int srv_create(const srv_config* cfg, void* stream, void* pool, size_t pool_bytes, srv_t** out) {
  if (!cfg || !out) return sfail(SIM_E_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 4096) return sfail(SIM_E_ARG, "max_slots must be in 1..4096");
  if (cfg->budget_bytes < kA) return sfail(SIM_E_ARG, "budget_bytes too small");
  if (cfg->arena_bytes && cfg->arena_bytes < kMinArena)
    return sfail(SIM_E_ARG, "arena_bytes must be 0 (default 64 MiB) or at least 1 MiB");
  if (cfg->grid > 65536) return sfail(SIM_E_ARG, "grid must be 0 (default 2048) or 1..65536");
  if (cfg->lane_workers > 64) return sfail(SIM_E_ARG, "lane_workers must be 0 (default 8) or 1..64");
  if (cfg->flags & ~(SRV_FLAG_NO_GRAPH | SRV_FLAG_U2_GLOBAL_INDEX | SRV_FLAG_NO_RP | SRV_FLAG_ONE_SEGMENT))
    return sfail(SIM_E_ARG, "unknown flags");
  std::unique_ptr<srv_t> s(new srv_t());
  s->cfg = *cfg;
  if (!s->cfg.arena_bytes) s->cfg.arena_bytes = 64ull << 20;
  s->grid = cfg->grid ? (int)cfg->grid : 2048;
  s->run_ops = cfg->max_run_ops ? cfg->max_run_ops : 4096u;
  s->lane_cap = cfg->lane_capacity == SRV_LANE_OFF ? 0 : cfg->lane_capacity;   // 0: no lane (default)
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  if (stream) {
    s->stream = static_cast<hipStream_t>(stream);
  } else {
    SRV_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->own_stream = true;
  }
  if (pool) {
    if (pool_bytes < cfg->budget_bytes) return sfail(SIM_E_NOMEM, "pool smaller than budget_bytes");
    s->pool_mem = static_cast<char*>(pool);
  } else {
    if (hipMalloc(&s->pool_mem, cfg->budget_bytes) != hipSuccess) return sfail(SIM_E_NOMEM, "pool allocation failed");
    s->own_pool = true;
  }
  s->pool.init(cfg->budget_bytes / kA * kA);
  const size_t ns = cfg->max_slots;
  SRV_HIP(hipMalloc(&s->d_ctl, ns * sizeof(SlotCtl)));
  SRV_HIP(mono_rp_init());
  SRV_HIP(hipMalloc(&s->d_rpctl, sizeof(Ctl)));
  {
    const Ctl zero{};
    SRV_HIP(hipMemcpy(s->d_rpctl, &zero, sizeof(Ctl), hipMemcpyHostToDevice));
  }
  SRV_HIP(hipHostMalloc(&s->h_ctl, ns * sizeof(SlotCtl)));
  for (int k = (int)ns - 1; k >= 0; --k) s->free_slots.push_back(k);
  // A tick has at most two first-round items per running request (a fused
  // run and the branching gate or measurement paired with it) and
  // n_mono + 3 n_u2 + n_meas + 5 <= 4 ns + 5 unit offsets for them; each of
  // the kMaxChain - 1 later measurement rounds adds at most one item per
  // request and ns + 1 unit offsets.
  s->max_items = (2 + (kMaxChain - 1)) * ns;
  s->max_units = (5 + (kMaxChain - 1)) * (ns + 1);
  s->items_off = al(sizeof(BTick));
  s->units_off = s->items_off + al(s->max_items * sizeof(BItem));
  s->chain_hdr_off = s->units_off + al(s->max_units * sizeof(uint32_t));
  s->arena_off = s->chain_hdr_off + al((kMaxChain - 1) * sizeof(BTick));
  s->tick_bytes = s->arena_off + s->cfg.arena_bytes;
  SRV_HIP(hipMalloc(&s->d_tick, s->tick_bytes));
  SRV_HIP(hipHostMalloc(&s->h_tick, s->tick_bytes));
  std::memset(s->h_tick, 0, s->arena_off);
  SRV_HIP(hipMemcpyAsync(s->d_tick, s->h_tick, s->arena_off, hipMemcpyHostToDevice, s->stream));
  SRV_HIP(hipStreamSynchronize(s->stream));
  int rc = capture_tick(s.get());
  if (rc) return rc;
  if (s->lane_cap) {
    const int nw = cfg->lane_workers ? (int)cfg->lane_workers : 8;
    s->lane_depth = nw + 1;
    srv_t* raw = s.get();
    for (int k = 0; k < nw; ++k) {
      hipStream_t st = nullptr;
      SRV_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->lane_streams.push_back(st);
      s->lane_threads.emplace_back([raw, st] { lane_main(raw, st); });
    }
  }
  {
    srv_t* raw = s.get();
    for (int k = 0; k < kBgThreads; ++k) s->bg_threads.emplace_back([raw] { bg_main(raw); });
  }
  *out = s.release();
  return SIM_OK;
}

int srv_destroy(srv_t* s) {
  if (!s) return SIM_OK;
  bg_shutdown(s);
  if (!s->lane_threads.empty()) {
    {
      std::lock_guard<std::mutex> lk(s->lane_mu);
      s->lane_stop = true;
      s->lane_todo.clear();   // requests running now finish; queued ones are dropped
    }
    s->lane_cv.notify_all();
    for (auto& t : s->lane_threads) t.join();
  }
  for (hipStream_t st : s->lane_streams) (void)hipStreamDestroy(st);
  (void)hipStreamSynchronize(s->stream);
  for (int m = 0; m < 16; ++m) {
    if (s->exec[m]) (void)hipGraphExecDestroy(s->exec[m]);
    if (s->graph[m]) (void)hipGraphDestroy(s->graph[m]);
  }
  if (s->d_tick) (void)hipFree(s->d_tick);
  if (s->h_tick) (void)hipHostFree(s->h_tick);
  if (s->d_ctl) (void)hipFree(s->d_ctl);
  if (s->d_rpctl) (void)hipFree(s->d_rpctl);
  if (s->h_ctl) (void)hipHostFree(s->h_ctl);
  if (s->own_pool && s->pool_mem) (void)hipFree(s->pool_mem);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return SIM_OK;
}

int srv_submit(srv_t* s, const sim_config* cfg, const sim_gate* gates, size_t n, sim_key basis, uint64_t* id) {
  if (!s || !cfg || !id || (n && !gates)) return sfail(SIM_E_ARG, "null argument");
  if (cfg->n_qubits < 1 || cfg->n_qubits > 128) return sfail(SIM_E_ARG, "n_qubits must be in 1..128");
  if (cfg->capacity < 1 || cfg->capacity >= (1ull << 31)) return sfail(SIM_E_ARG, "capacity out of range");
  if (!(cfg->eps >= 0.0) || !std::isfinite(cfg->eps)) return sfail(SIM_E_ARG, "eps must be finite and >= 0");
  if (cfg->mono_mode > SIM_MONO_BITSLICE) return sfail(SIM_E_ARG, "unknown mono_mode");
  if (!key_fits(cfg->n_qubits, basis.lo, basis.hi)) return sfail(SIM_E_ARG, "basis has bits above n_qubits");
  std::unique_ptr<Request> r(new Request());
  r->cfg = *cfg;
  r->cfg.load_factor = lf_or_default(cfg->load_factor);
  if (!(r->cfg.load_factor > 0.0 && r->cfg.load_factor <= 0.9)) return sfail(SIM_E_ARG, "load_factor out of range");
  r->large = s->lane_cap && cfg->capacity >= s->lane_cap;
  if (r->large) {
    r->fp = Footprint{};
    r->fp.total = al(sim_workspace_bytes(&r->cfg));
    if (r->fp.total == 0) return sfail(SIM_E_ARG, "invalid configuration for the large-state lane");
  } else {
    r->fp = footprint_of(r->cfg, r->cfg.load_factor);
  }
  if (r->fp.total > s->pool.size) return sfail(SIM_E_CAPACITY, "request footprint exceeds the pool");
  r->basis = basis;
  // Copy and validate on the host thread pool; the first invalid op is reported.
  r->gates.resize(n);
  std::vector<size_t> bad(HostPool::kMaxThreads, SIZE_MAX);
  parallel_parts(n, 16384, [&](size_t b, size_t e, size_t p) {
    std::memcpy(r->gates.data() + b, gates + b, (e - b) * sizeof(sim_gate));
    std::string ignored;
    for (size_t i = b; i < e; ++i)
      if (!gate_valid(cfg->n_qubits, gates[i], &ignored)) {
        bad[p] = i;
        break;
      }
  });
  const size_t first_bad = *std::min_element(bad.begin(), bad.end());
  if (first_bad != SIZE_MAX) {
    std::string why;
    gate_valid(cfg->n_qubits, gates[first_bad], &why);
    return sfail(SIM_E_ARG, "op " + std::to_string(first_bad) + ": " + why);
  }
  r->id = s->next_id++;
  *id = r->id;
  (r->large ? s->lane_queue : s->queue).push_back(r->id);
  Request* raw = r.get();
  s->reqs[r->id] = std::move(r);
  s->stats.submitted++;
  if (!raw->large) bg_push(s, raw, BG_COMPILE);
  return SIM_OK;
}

namespace {
double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// After a tick is launched, each request in it has the grouping of the fused
// run it is expected to take next made in the background.  Its state size
// after the tick is predicted (unchanged by a fused run or, as an upper bound,
// by a measurement; doubled, up to the capacity, by a branching gate), which
// fixes the cap's skip decisions and with them where the run ends.  A later
// tick uses the grouping only if the run that comes is the same, so a wrong
// prediction costs time, not results.
void group_ahead(srv_t* s, const std::vector<Request*>& mono, const std::vector<Request*>& u2,
                 const std::vector<Request*>& meas) {
  auto plan = [&](Request* r, uint64_t nnz) {
    Cursor c{r->i, r->mono_seen, 0};
    size_t b = 0, len = 0, op = 0;
    if (scan_segment(s, *r, nnz, c, &b, &len, &op) != SEG_MONO) return;
    BsRun br{};
    if (!r->rc.run_params(b, len, r->cfg.mono_mode, r->cfg.bs_min_gates, &br)) return;
    r->ahead.valid = false;
    r->ahead.b = b;
    r->ahead.len = len;
    r->ahead.rp = use_rp(s, nnz);
    r->ahead.br = br;
    r->ahead.grp.clear();
    r->ahead.prog.clear();
    bg_push(s, r, BG_GROUP);
  };
  for (Request* r : mono) plan(r, r->nnz);
  for (Request* r : meas) plan(r, r->nnz);
  for (Request* r : u2) plan(r, std::min<uint64_t>(2 * r->nnz, r->cfg.capacity));
}

// Finished requests whose states have been copied out release their memory
// and become done.
int fold_copies(srv_t* s) {
  for (size_t k = 0; k < s->copying.size();) {
    Request* r = s->copying[k];
    if (r->bg_busy.load(std::memory_order_acquire)) {
      ++k;
      continue;
    }
    if (r->copy_err != hipSuccess)
      return sfail(SIM_E_HIP, std::string("copying a finished state out: ") + hipGetErrorString(r->copy_err));
    const int rc = finish(s, *r, SRV_DONE, SIM_OK);
    if (rc) return rc;
    s->copying[k] = s->copying.back();
    s->copying.pop_back();
  }
  return SIM_OK;
}
}  // namespace

int srv_tick(srv_t* s, uint32_t* running, uint32_t* queued) {
  if (!s) return sfail(SIM_E_ARG, "null handle");
  const auto t_tick = std::chrono::steady_clock::now();
  const double wait0 = s->stats.wait_ms;
  struct HostTime {
    srv_t* s;
    std::chrono::steady_clock::time_point t0;
    double wait0;
    ~HostTime() { s->stats.host_ms += ms_since(t0) - (s->stats.wait_ms - wait0); }
  } host_time{s, t_tick, wait0};
  lane_fold(s);
  int rc = fold_copies(s);
  if (rc) return rc;
  rc = admit(s);
  if (rc) return rc;
  // Assemble the work list.
  auto* hdr = reinterpret_cast<BTick*>(s->h_tick);
  auto* items = reinterpret_cast<BItem*>(s->h_tick + s->items_off);
  auto* units = reinterpret_cast<uint32_t*>(s->h_tick + s->units_off);
  char* arena = s->h_tick + s->arena_off;
  size_t arena_used = 0;
  std::vector<Request*> mono, u2, meas;
  std::vector<BItem> mono_items, u2_items, meas_items, u2s_items;
  std::vector<Request*> done_now;
  // Every request's next segment; the fused runs that take the bit-sliced
  // form are grouped on the host thread pool, one request per task (runs of
  // different requests are independent).
  struct Seg {
    Request* r;
    SegKind k;
    size_t b = 0, len = 0, op = 0;
    bool bsl = false;
    bool rp = false;     // bit-sliced run on the register-plane kernel (prog), else groups
    BsRun br{};
    std::vector<BsGroup> grp;
    std::vector<RpRec> prog;
  };
  // Register-plane runs of this tick: (request, arena offset, records, run).
  struct RpItem {
    Request* r;
    size_t off;
    uint32_t nrec;
    BsRun br;
  };
  std::vector<RpItem> rp_items;
  std::vector<Seg> segs;
  segs.reserve(s->running.size());
  std::vector<size_t> to_group;
  // Requests whose fused run was deferred last tick (the arena was full) go
  // first, so that none waits more than one tick for arena space.
  std::stable_partition(s->running.begin(), s->running.end(), [](const Request* r) { return r->deferred; });
  size_t waiting = 0;   // requests whose background job (compile, grouping) is not done
  for (Request* r : s->running) {
    if (r->bg_busy.load(std::memory_order_acquire)) {
      ++waiting;
      continue;
    }
    Seg sg{r, SEG_NONE};
    sg.k = next_segment(s, *r, &sg.b, &sg.len, &sg.op);
    r->seg = sg.k;
    if (sg.k == SEG_NONE) {
      done_now.push_back(r);
      continue;
    }
    if (sg.k == SEG_MONO) {
      sg.bsl = r->rc.run_params(sg.b, sg.len, r->cfg.mono_mode, r->cfg.bs_min_gates, &sg.br);
      if (sg.bsl) {
        sg.rp = use_rp(s, r->nnz);
        // group() and schedule() depend only on the run, so a grouping or
        // program made ahead for the same run is the one they would make now.
        if (r->ahead.valid && r->ahead.b == sg.b && r->ahead.len == sg.len && r->ahead.rp == sg.rp) {
          sg.grp = std::move(r->ahead.grp);
          sg.prog = std::move(r->ahead.prog);
          sg.br = r->ahead.br;
          s->stats.ahead_hits++;
        } else {
          to_group.push_back(segs.size());
        }
      }
    }
    r->ahead.valid = false;
    r->ahead.grp.clear();
    r->ahead.prog.clear();
    segs.push_back(std::move(sg));
  }
  {
    const auto t_g = std::chrono::steady_clock::now();
    HostPool::get().run(to_group.size(), [&](size_t t) {
      Seg& sg = segs[to_group[t]];
      if (sg.rp) sg.r->rc.schedule(sg.b, sg.len, sg.prog, &sg.br);
      else sg.r->rc.group(sg.b, sg.len, sg.grp, &sg.br);
    });
    s->stats.group_ms += ms_since(t_g);
  }
  // An item of r on its current buffers (the segment fields left empty).
  auto base_item = [&](Request* r) {
    BItem it{};
    it.in = r->buf[r->cur];
    it.out = r->buf[r->cur ^ 1];
    it.ctl = s->d_ctl + r->slot;
    it.other = (uint32_t)(r->cur ^ 1);
    it.wide = r->cfg.n_qubits > 64 ? 1u : 0u;
    it.nnz = r->nnz;
    it.cap = r->cfg.capacity;
    return it;
  };
  // Requests whose measurement this tick has later steps (a chain).
  std::vector<Request*> chains;
  // The measurement item of step j of r's chain (base: r's current buffers).
  auto meas_item = [&](Request* r, BItem it, uint32_t j) {
    if (j & 1u) {
      std::swap(it.in, it.out);
      it.other ^= 1u;
    }
    const sim_gate& g = r->gates[r->chain_op[j]];
    it.chain = j;
    it.q = g.target;
    it.forced = g.forced;
    it.u = g.u;
    it.part = r->part;
    it.cnt1 = r->cnt1;
    it.tot = r->tot;
    return it;
  };
  // A branching gate or measurement item of r (the gate at op index op).
  auto add_gate = [&](Request* r, BItem it, SegKind k, size_t op) {
    const sim_gate& g = r->gates[op];
    if (k == SEG_U2) {
      it.u2 = u2_desc(g, r->cfg.eps);
      const uint64_t slots = std::min<uint64_t>(index_slots(r->nnz, r->cfg.load_factor), r->fp.slots);
      it.table = r->table;
      it.mask = slots - 1;
      it.partner = r->partner;
      it.tot = r->tot;
      r->st.updates += r->nnz;
      u2.push_back(r);
      // Small states take the one-block kernel with the index in LDS.
      const bool small = r->nnz <= kLdsU2Max && !(s->cfg.flags & SRV_FLAG_U2_GLOBAL_INDEX);
      (small ? u2s_items : u2_items).push_back(it);
    } else {
      // Measurements right after this one run in later rounds of the tick:
      // each needs only the previous one's output, whose entry count the
      // kernels read on the device.
      r->chain_len = 1;
      r->chain_op[0] = op;
      if (!(s->cfg.flags & SRV_FLAG_ONE_SEGMENT))
        while (r->chain_len < kMaxChain && r->i < r->gates.size() && r->gates[r->i].op == SIM_OP_MEASURE)
          r->chain_op[r->chain_len++] = r->i++;
      if (r->chain_len > 1) {
        chains.push_back(r);
        s->stats.chained += r->chain_len - 1;
      }
      meas.push_back(r);
      meas_items.push_back(meas_item(r, it, 0));
    }
  };
  // A branching gate or measurement that comes right after a fused run joins
  // the run's tick: the run works in place and keeps the entry count (so the
  // cap's skip decisions before the gate are the ones the next tick would
  // make), register-plane runs go before the graph, and the graph runs the
  // fused kernels before the branching and measurement kernels.  What is
  // paired depends on the request alone; its kernels and their inputs are
  // those of two ticks, so results are unchanged.
  auto pair_gate = [&](Request* r, const BItem& base) {
    if (s->cfg.flags & SRV_FLAG_ONE_SEGMENT) return false;
    Cursor c{r->i, r->mono_seen, 0};
    size_t b2 = 0, len2 = 0, op2 = 0;
    const SegKind k2 = scan_segment(s, *r, r->nnz, c, &b2, &len2, &op2);
    if (k2 != SEG_U2 && k2 != SEG_MEAS) return false;
    r->i = c.i;
    r->mono_seen = c.mono_seen;
    r->st.u2_skipped += c.skipped;
    add_gate(r, base, k2, op2);
    s->stats.paired++;
    return true;
  };
  for (Seg& sg : segs) {
    Request* r = sg.r;
    const SegKind k = sg.k;
    size_t b = sg.b, len = sg.len;
    const size_t op = sg.op;
    BItem it = base_item(r);
    if (k == SEG_MONO) {
      const BItem base = it;
      const bool bsl = sg.bsl;
      uint32_t flags = 0;
      for (size_t q = b; q < b + len; ++q) {
        if (r->rc.descs[q].flags & kHasPhase) flags |= kRunPhase;
        if (r->rc.descs[q].flags & kFlip) flags |= kRunFlip;
      }
      it.run_flags = flags;
      // The run's ops go into the tick's arena.  A run that does not fit what
      // is left is deferred whole to the next tick (never cut: that would
      // change its rounding); every run fits an empty arena (arena_run_cap).
      const size_t bytes = !bsl ? len * sizeof(MonoDesc)
                           : sg.rp ? sg.prog.size() * sizeof(RpRec)
                                   : sg.grp.size() * sizeof(BsGroup);
      r->deferred = arena_used + al(bytes) > s->cfg.arena_bytes;
      if (r->deferred) {
        // Give back the run's ops: they are re-read next tick (skip decisions
        // there depend only on nnz, which is unchanged), and so is the run,
        // whose grouping is kept for it.
        const size_t back_to = r->mono_op[b];
        for (size_t q = back_to; q < r->i; ++q)
          if (r->gates[q].op == SIM_OP_U2) r->st.u2_skipped--;
        r->i = back_to;
        r->mono_seen = b;
        if (bsl) {
          r->ahead.valid = true;
          r->ahead.b = b;
          r->ahead.len = len;
          r->ahead.rp = sg.rp;
          r->ahead.br = sg.br;
          r->ahead.grp = std::move(sg.grp);
          r->ahead.prog = std::move(sg.prog);
        }
        continue;
      }
      r->st.updates += r->nnz * len;
      r->st.mono_passes++;
      if (bsl) {
        r->st.bitslice_passes++;
        s->stats.bitslice_runs++;
      }
      if (bsl && sg.rp) {
        // Its own launch ahead of the graph; the request has no item in it.
        std::memcpy(arena + arena_used, sg.prog.data(), bytes);
        rp_items.push_back(RpItem{r, arena_used, (uint32_t)sg.prog.size(), sg.br});
        arena_used += al(bytes);
        s->stats.rp_runs++;
      } else {
        if (bsl) {
          std::memcpy(arena + arena_used, sg.grp.data(), bytes);
          it.gops = reinterpret_cast<const BsGroup*>(s->d_tick + s->arena_off + arena_used);
          it.ngroups = (uint32_t)sg.grp.size();
          it.run = sg.br;
        } else {
          std::memcpy(arena + arena_used, r->rc.descs.data() + b, bytes);
          it.dops = reinterpret_cast<const MonoDesc*>(s->d_tick + s->arena_off + arena_used);
          it.n_dops = (uint32_t)len;
        }
        arena_used += al(bytes);
        mono_items.push_back(it);
      }
      if (!pair_gate(r, base)) mono.push_back(r);
    } else {
      add_gate(r, it, k, op);
    }
  }
  // Finished requests leave the tick; their states are copied out in the
  // background (their memory is released once that is done).
  for (Request* r : done_now) {
    s->running.erase(std::find(s->running.begin(), s->running.end(), r));
    s->copying.push_back(r);
    bg_push(s, r, BG_COPY);
  }
  const uint32_t nm = (uint32_t)mono_items.size(), nu = (uint32_t)u2_items.size(), nq = (uint32_t)meas_items.size();
  const uint32_t ns = (uint32_t)u2s_items.size();
  const uint32_t nrp = (uint32_t)rp_items.size();
  // Later measurement rounds: round j holds step j of every chain longer
  // than j (the count before the chain bounds its units).
  uint32_t rounds = 1;
  for (const Request* r : chains) rounds = std::max(rounds, r->chain_len);
  std::vector<std::vector<BItem>> later(rounds - 1);
  for (Request* r : chains)
    for (uint32_t j = 1; j < r->chain_len; ++j) later[j - 1].push_back(meas_item(r, base_item(r), j));
  size_t n_later = 0, later_units = 0;
  for (const auto& v : later) {
    n_later += v.size();
    later_units += v.size() + 1;
  }
  if (nm + nu + nq + ns + nrp) {
    const size_t n_units = (size_t)nm + 3 * (size_t)nu + nq + 5;
    if ((size_t)nm + nu + nq + ns + n_later > s->max_items || n_units + later_units > s->max_units)
      return sfail(SIM_E_NOMEM, "tick work list exceeds its area");
    std::memset(hdr, 0, sizeof(BTick));
    hdr->n_mono = nm;
    hdr->n_u2 = nu;
    hdr->n_meas = nq;
    hdr->n_u2s = ns;
    uint32_t w = 0;
    auto prefix = [&](uint32_t* at, const std::vector<BItem>& v, auto units_of) {
      uint32_t acc = 0;
      for (size_t k = 0; k < v.size(); ++k) {
        at[k] = acc;
        acc += units_of(v[k]);
      }
      at[v.size()] = acc;
    };
    auto chunks = [](const BItem& it) { return (uint32_t)((it.nnz + kChunk - 1) / kChunk); };
    hdr->mono_u0 = w;
    prefix(units + w, mono_items, chunks);
    w += nm + 1;
    hdr->fill_u0 = w;
    prefix(units + w, u2_items, [](const BItem& it) { return (uint32_t)((it.mask + kFillUnit) / kFillUnit); });
    w += nu + 1;
    hdr->build_u0 = w;
    prefix(units + w, u2_items, chunks);
    w += nu + 1;
    hdr->chunk_u0 = w;
    prefix(units + w, u2_items, chunks);
    w += nu + 1;
    hdr->meas_u0 = w;
    prefix(units + w, meas_items, chunks);
    w += nq + 1;
    size_t ni = 0;
    for (const auto& v : {&mono_items, &u2_items, &meas_items, &u2s_items})
      for (const BItem& it : *v) items[ni++] = it;
    // Each later round: its header (only measurement items), first-unit
    // array and items after everything before it.
    std::vector<size_t> later_i0(later.size());
    auto* later_hdr = reinterpret_cast<BTick*>(s->h_tick + s->chain_hdr_off);
    for (size_t j = 0; j < later.size(); ++j) {
      std::memset(&later_hdr[j], 0, sizeof(BTick));
      later_hdr[j].n_meas = (uint32_t)later[j].size();
      later_hdr[j].meas_u0 = w;
      prefix(units + w, later[j], chunks);
      w += (uint32_t)later[j].size() + 1;
      later_i0[j] = ni;
      for (const BItem& it : later[j]) items[ni++] = it;
    }
    SRV_HIP(hipMemcpyAsync(s->d_tick, s->h_tick, s->items_off + ni * sizeof(BItem), hipMemcpyHostToDevice,
                           s->stream));
    if (!later.empty())
      SRV_HIP(hipMemcpyAsync(s->d_tick + s->chain_hdr_off, later_hdr, later.size() * sizeof(BTick),
                             hipMemcpyHostToDevice, s->stream));
    SRV_HIP(hipMemcpyAsync(s->d_tick + s->units_off, units, w * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
    if (arena_used)
      SRV_HIP(hipMemcpyAsync(s->d_tick + s->arena_off, arena, arena_used, hipMemcpyHostToDevice, s->stream));
    // Register-plane runs first, on the same stream: each finishes before the
    // graph's kernels start, and no two run at once.
    for (const RpItem& x : rp_items) {
      Request* r = x.r;
      const int grid = (int)std::max<uint64_t>(1, (r->nnz + 2047) / 2048);
      launch_mono_rp(s->stream, r->buf[r->cur], &s->d_ctl[r->slot].nnz[r->cur],
                     reinterpret_cast<const RpRec*>(s->d_tick + s->arena_off + x.off), x.nrec, x.br, s->d_rpctl, grid);
      SRV_HIP(hipGetLastError());
    }
    // Only the kernel families that have items this tick.
    const uint32_t fam = (nm ? kFamMono : 0u) | (nu ? kFamU2 : 0u) | (ns ? kFamU2s : 0u) | (nq ? kFamMeas : 0u);
    if (fam == 0) {
      // only register-plane runs this tick
    } else if (s->exec[fam]) {
      SRV_HIP(hipGraphLaunch(s->exec[fam], s->stream));
    } else {
      launch_batch_tick(s->stream, reinterpret_cast<const BTick*>(s->d_tick),
                        reinterpret_cast<const BItem*>(s->d_tick + s->items_off),
                        reinterpret_cast<const uint32_t*>(s->d_tick + s->units_off), s->grid, fam);
      SRV_HIP(hipGetLastError());
    }
    // Later measurement rounds, in order, after the graph.
    for (size_t j = 0; j < later.size(); ++j) {
      launch_batch_meas(s->stream, reinterpret_cast<const BTick*>(s->d_tick + s->chain_hdr_off) + j,
                        reinterpret_cast<const BItem*>(s->d_tick + s->items_off) + later_i0[j],
                        reinterpret_cast<const uint32_t*>(s->d_tick + s->units_off), s->grid);
      SRV_HIP(hipGetLastError());
    }
    int max_slot = -1;
    for (Request* r : s->running) max_slot = std::max(max_slot, r->slot);
    SRV_HIP(hipMemcpyAsync(s->h_ctl, s->d_ctl, (size_t)(max_slot + 1) * sizeof(SlotCtl), hipMemcpyDeviceToHost,
                           s->stream));
    // The expected next runs are grouped in the background while the tick runs.
    {
      const auto t_a = std::chrono::steady_clock::now();
      group_ahead(s, mono, u2, meas);
      s->stats.ahead_ms += ms_since(t_a);
    }
    {
      const auto t_w = std::chrono::steady_clock::now();
      SRV_HIP(hipStreamSynchronize(s->stream));
      s->stats.wait_ms += ms_since(t_w);
    }
    s->stats.ticks++;
    s->stats.items += nm + nu + nq + ns + nrp + n_later;
    // Fold the results back.
    std::vector<std::pair<Request*, int>> failed;
    for (Request* r : u2) {
      const SlotCtl& c = s->h_ctl[r->slot];
      if (c.status & kStOverflow) {
        failed.emplace_back(r, SIM_E_CAPACITY);
        continue;
      }
      r->cur ^= 1;
      r->nnz = c.nnz[r->cur];
      r->st.u2_applied++;
      r->st.peak_nnz = std::max<uint64_t>(r->st.peak_nnz, r->nnz);
    }
    for (Request* r : meas) {
      // Outcomes up to the first zero-probability one (which fails the
      // request, as it would have alone).
      const SlotCtl& c = s->h_ctl[r->slot];
      uint32_t k = 0;
      for (; k < r->chain_len && c.chain_out[k] >= 0; ++k) {
        r->outcomes.push_back(c.chain_out[k]);
        r->st.measures++;
      }
      if (k < r->chain_len || (c.status & kStMeasure)) {
        failed.emplace_back(r, SIM_E_STATE);
        continue;
      }
      r->cur ^= (int)(r->chain_len & 1u);
      r->nnz = c.nnz[r->cur];
    }
    for (auto& f : failed) {
      bg_wait(s, f.first);   // a grouping made for it may be in flight
      rc = finish(s, *f.first, SRV_FAILED, f.second);
      if (rc) return rc;
      s->running.erase(std::find(s->running.begin(), s->running.end(), f.first));
    }
  }
  rc = fold_copies(s);
  if (rc) return rc;
  if (nm + nu + nq + ns + nrp == 0 && (waiting || !s->copying.empty())) {
    // Nothing launched: wait (briefly) for the background work instead of spinning.
    const auto t_w = std::chrono::steady_clock::now();
    bg_wait_any(s, 200);
    s->stats.wait_ms += ms_since(t_w);
  }
  if (s->running.empty() && s->lane_in_flight) {
    // Nothing batched to do: wait (briefly) for the lane instead of spinning.
    const auto t_w = std::chrono::steady_clock::now();
    std::unique_lock<std::mutex> lk(s->lane_mu);
    s->lane_done_cv.wait_for(lk, std::chrono::microseconds(200), [&] { return !s->lane_done.empty(); });
    lk.unlock();
    s->stats.wait_ms += ms_since(t_w);
  }
  if (running) *running = (uint32_t)(s->running.size() + s->copying.size() + s->lane_in_flight);
  if (queued) *queued = (uint32_t)(s->queue.size() + s->lane_queue.size());
  s->stats.pool_peak_bytes = s->pool.peak;
  s->stats.pool_used_bytes = s->pool.used;
  return SIM_OK;
}

int srv_run(srv_t* s) {
  if (!s) return sfail(SIM_E_ARG, "null handle");
  uint32_t run = 1, q = 1;
  while (run || q) {
    // A tick that starts with nothing running has the whole pool and every
    // slot free: if it admits nothing, the queue's head can never fit.
    const bool idle = s->running.empty() && s->copying.empty() && s->lane_in_flight == 0;
    const uint64_t before = s->stats.admitted;
    int rc = srv_tick(s, &run, &q);
    if (rc) return rc;
    if (idle && q && s->stats.admitted == before) return sfail(SIM_E_NOMEM, "queued request can never be admitted");
  }
  return SIM_OK;
}

int srv_poll(srv_t* s, uint64_t id, int32_t* state, int32_t* error) {
  if (!s || !state) return sfail(SIM_E_ARG, "null argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(SIM_E_ARG, "unknown request id");
  *state = it->second->state;
  if (error) *error = it->second->error;
  return SIM_OK;
}

namespace {
// The finished request id, or an error.
int done_request(srv_t* s, uint64_t id, Request** out) {
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(SIM_E_ARG, "unknown request id");
  Request& r = *it->second;
  if (r.state != SRV_DONE) return sfail(r.state == SRV_FAILED ? r.error : SIM_E_STATE, "request not done");
  *out = &r;
  return SIM_OK;
}

int result_rest(Request& r, uint64_t cap, uint64_t* nnz, int32_t* outcomes, uint64_t out_cap, uint64_t* n_out,
                sim_stats* stats) {
  *nnz = r.res_n;
  if (n_out) *n_out = r.outcomes.size();
  if (stats) *stats = r.st;
  if (cap < r.res_n || (outcomes && out_cap < r.outcomes.size())) return sfail(SIM_E_BUFFER, "buffer too small");
  if (outcomes && !r.outcomes.empty()) std::memcpy(outcomes, r.outcomes.data(), r.outcomes.size() * 4);
  return SIM_OK;
}
}  // namespace

int srv_result(srv_t* s, uint64_t id, sim_key* keys, sim_c64* amps, uint64_t cap, uint64_t* nnz, int32_t* outcomes,
               uint64_t out_cap, uint64_t* n_out, sim_stats* stats) {
  if (!s || !nnz) return sfail(SIM_E_ARG, "null argument");
  Request* r = nullptr;
  int rc = done_request(s, id, &r);
  if (rc) return rc;
  rc = result_rest(*r, cap, nnz, outcomes, out_cap, n_out, stats);
  if (rc) return rc;
  const uint64_t* lo = r->res_lo.get();
  const uint64_t* hi = r->res_hi.get();
  const sim_c64* a = r->res_amp.get();
  parallel_parts(r->res_n, 1u << 16, [&](size_t b, size_t e, size_t) {
    if (keys)
      for (size_t k = b; k < e; ++k) keys[k] = sim_key{lo[k], hi ? hi[k] : 0};
    if (amps) std::memcpy(amps + b, a + b, (e - b) * sizeof(sim_c64));
  });
  return SIM_OK;
}

int srv_result_soa(srv_t* s, uint64_t id, uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps, uint64_t cap,
                   uint64_t* nnz, int32_t* outcomes, uint64_t out_cap, uint64_t* n_out, sim_stats* stats) {
  if (!s || !nnz) return sfail(SIM_E_ARG, "null argument");
  Request* r = nullptr;
  int rc = done_request(s, id, &r);
  if (rc) return rc;
  rc = result_rest(*r, cap, nnz, outcomes, out_cap, n_out, stats);
  if (rc) return rc;
  const uint64_t* lo = r->res_lo.get();
  const uint64_t* hi = r->res_hi.get();
  const sim_c64* a = r->res_amp.get();
  parallel_parts(r->res_n, 1u << 16, [&](size_t b, size_t e, size_t) {
    if (key_lo) std::memcpy(key_lo + b, lo + b, (e - b) * 8);
    if (key_hi) {
      if (hi) std::memcpy(key_hi + b, hi + b, (e - b) * 8);
      else std::memset(key_hi + b, 0, (e - b) * 8);
    }
    if (amps) std::memcpy(amps + b, a + b, (e - b) * sizeof(sim_c64));
  });
  return SIM_OK;
}

int srv_release(srv_t* s, uint64_t id) {
  if (!s) return sfail(SIM_E_ARG, "null handle");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(SIM_E_ARG, "unknown request id");
  if (it->second->state == SRV_QUEUED || it->second->state == SRV_RUNNING)
    return sfail(SIM_E_STATE, "request still queued or running");
  s->reqs.erase(it);
  return SIM_OK;
}

int srv_get_stats(srv_t* s, srv_stats* out) {
  if (!s || !out) return sfail(SIM_E_ARG, "null argument");
  {
    std::lock_guard<std::mutex> lk(s->bg_mu);
    s->stats.copy_ms = s->bg_copy_ms;
  }
  *out = s->stats;
  return SIM_OK;
}

const char* srv_last_error(void) { return g_srv_error.c_str(); }

}  // extern "C"
