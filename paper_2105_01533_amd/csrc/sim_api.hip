// Host engine and C-ABI of libsparsesim (see include/sparsesim.h).
//
// The engine walks the op list once.  Phase/permutation ops accumulate into a
// pending run that is launched as one fused pass (Sec. 3.2); a branching op
// with a cap is decided against the exact entry count, which phase/permutation
// runs never change, so skipped branching ops do not end a run.  The entry
// count lives on the device; the host keeps an upper bound and reads the
// exact value only when a cap decision or the capacity check needs it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sparsesim.h"
#include "host_pool.h"
#include "run_compiler.h"
#include "sim_internal.h"

using namespace sparsesim;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

// The thread's last error, for the library's other host sources.
int sparsesim::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(SIM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint64_t table_slots(uint64_t n, double lf) {
  const uint64_t want = (uint64_t)std::ceil((double)(n ? n : 1) / lf) + 1;
  return std::max<uint64_t>(64, next_pow2(want));
}

struct Layout {
  size_t buf_lo[2], buf_hi[2], buf_amp[2];
  size_t table, partner, tot, tot2, status, cnt1, part, ctl, total;
  uint64_t slots;
};

bool config_ok(const sim_config* c, std::string* why) {
  if (!c) return *why = "null config", false;
  if (c->n_qubits < 1 || c->n_qubits > 128) return *why = "n_qubits must be in 1..128", false;
  if (c->capacity < 1 || c->capacity >= (1ull << 31)) return *why = "capacity must be in 1..2^31-1", false;
  if (!(c->eps >= 0.0) || !std::isfinite(c->eps)) return *why = "eps must be finite and >= 0", false;
  if (c->load_factor != 0.0 && !(c->load_factor > 0.0 && c->load_factor <= 0.9))
    return *why = "load_factor must be in (0, 0.9]", false;
  if (c->block != 0 && c->block != 64 && c->block != 128 && c->block != 256)
    return *why = "block must be 64, 128 or 256", false;
  if (c->flags & ~(SIM_FLAG_U2_TWO_PASS | SIM_FLAG_BS_LDS | SIM_FLAG_U2_GLOBAL_INDEX | SIM_FLAG_COUNT_INDEX |
                   SIM_FLAG_NO_UNIFORM))
    return *why = "unknown flags", false;
  if (c->mono_mode > SIM_MONO_BITSLICE) return *why = "unknown mono_mode", false;
  return true;
}

double lf_of(const sim_config* c) { return c->load_factor > 0.0 ? c->load_factor : 0.5; }

Layout layout_of(const sim_config* c) {
  Layout L{};
  const uint64_t cap = c->capacity;
  const bool wide = c->n_qubits > 64;
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    L.buf_lo[b] = off;
    off += align_up(cap * 8);
    L.buf_hi[b] = wide ? off : (size_t)-1;
    if (wide) off += align_up(cap * 8);
    L.buf_amp[b] = off;
    off += align_up(cap * 16);
  }
  L.slots = table_slots(cap, lf_of(c));
  L.table = off;
  off += align_up(L.slots * 8);
  L.partner = off;
  off += align_up(cap * 4);
  L.tot = off;
  off += align_up(kMaxBlocks * 4);
  L.tot2 = off;
  off += align_up(kMaxBlocks * 4);
  L.status = off;
  off += align_up(kMaxBlocks * 8);
  L.cnt1 = off;
  off += align_up(kMaxBlocks * 4);
  L.part = off;
  off += align_up(kMaxBlocks * 16);
  L.ctl = off;
  off += align_up(sizeof(Ctl));
  L.total = off;
  return L;
}

template <typename T>
struct DevVec {            // library-owned growable device array
  T* p = nullptr;
  size_t n = 0;
  hipError_t reserve(size_t want) {
    if (want <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    const size_t m = std::max<size_t>(want, 256);
    hipError_t e = hipMalloc(&p, m * sizeof(T));
    if (e == hipSuccess) n = m;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Pinned host staging for asynchronous uploads, shared by all handles of the
// process: a call borrows buffers and gives them back when it returns (after
// its stream has drained, so no copy in flight still reads them).  Handles
// that come and go -- one per request -- then pay no pinned allocation.
class PinnedPool {
 public:
  static PinnedPool& get() {
    static PinnedPool pool;
    return pool;
  }
  // A buffer of at least `bytes`, or nullptr if the allocation fails.
  void* take(size_t bytes, size_t* got) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t k = 0; k < free_.size(); ++k)
        if (free_[k].second >= bytes) {
          auto e = free_[k];
          free_.erase(free_.begin() + (long)k);
          *got = e.second;
          return e.first;
        }
    }
    const size_t m = std::max<size_t>(bytes + bytes / 4, 1u << 16);
    void* p = nullptr;
    if (hipHostMalloc(&p, m) != hipSuccess) return nullptr;
    *got = m;
    return p;
  }
  void give(void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace_back(p, bytes);
  }

 private:
  std::mutex mu_;
  std::vector<std::pair<void*, size_t>> free_;
};

// Staging borrowed for one call: grown on demand (growth drains the stream
// first), returned to the pool with the stream drained.
template <class T>
struct Staging {
  hipStream_t st;
  T* p = nullptr;
  size_t bytes = 0;
  explicit Staging(hipStream_t s) : st(s) {}
  hipError_t reserve(size_t n) {
    if (n * sizeof(T) <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) return e;
      PinnedPool::get().give(p, bytes);
      p = nullptr;
      bytes = 0;
    }
    p = static_cast<T*>(PinnedPool::get().take(n * sizeof(T), &bytes));
    return p ? hipSuccess : hipErrorOutOfMemory;
  }
  ~Staging() {
    if (!p) return;
    (void)hipStreamSynchronize(st);
    PinnedPool::get().give(p, bytes);
  }
};

}  // namespace

// Kernel classes timed by the profiler.
// Host classes (wall clock, always measured): validation and op compilation
// at the start of a call, grouping of bit-sliced runs, and time blocked in
// stream synchronisations.
enum KClass { KC_MONO = 0, KC_FILL, KC_BUILD, KC_U2_PROBE, KC_U2_COUNT, KC_SCAN, KC_U2_WRITE, KC_M_REDUCE,
              KC_M_DECIDE, KC_M_WRITE, KC_U2_LDS, KC_KERNELS, KC_H_PREPARE = KC_KERNELS, KC_H_GROUP, KC_H_SYNC,
              KC_COUNT };
static const char* const kClassNames[KC_COUNT] = {"mono_pass", "index_fill", "index_build", "u2_probe", "u2_count",
                                                  "block_scan", "u2_write", "measure_reduce", "measure_decide",
                                                  "measure_write", "u2_lds", "host_prepare", "host_group",
                                                  "host_sync"};

struct sim_t {
  sim_config cfg;
  // Qubits whose bit is the same in every entry (host-side, exact for the
  // states it is set from and kept conservatively: a bit leaves the set on any
  // gate that could make it differ between entries).  A branching gate whose
  // partner mask meets the set has no partners (run_u2's split).
  uint64_t uni_lo = ~0ull, uni_hi = ~0ull;
  // profiling
  uint32_t profile = 0;          // bit c: kernel class c is timed with events
  bool no_alloc = false;         // inside sim_apply_gates_static: no events, threads or allocations
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_pending;   // (class, index of start event)
  uint64_t k_launches[KC_COUNT] = {};
  double k_ms[KC_COUNT] = {};
  uint64_t mono_bytes_base = 0, mono_updates = 0;
  uint64_t pass_bytes_base[5] = {};
  // Single-pass branching kernel: tile status words, the launch epoch and the
  // tile counter's value at the start of the next launch.
  uint64_t* status = nullptr;
  uint32_t u2_epoch = 0;
  uint32_t ticket_base = 0;
  // Hash index slots [0, table_dirty) may hold entries; the rest are empty
  // (the whole index is emptied at creation).  The single-pass branching
  // kernel empties the slots its gate used, so a separate clearing launch is
  // needed only after the two-pass form.
  uint64_t table_dirty = 0;
  // Sums of a qubit formed by the last measurement's write (see run_measure);
  // valid only until the next operation.
  struct {
    bool valid;
    uint32_t q;
    int grid;
    const uint32_t* off;
  } mchain = {false, 0, 0, nullptr};
  hipStream_t stream;
  int device;                  // the device current at creation
  bool wide;
  char* ws;
  bool ws_owned;
  Layout L;
  Buf buf[2];
  int cur;
  uint64_t* table;
  uint32_t* partner;
  BlockScratch bs;
  Ctl* ctl;
  uint64_t* h_pinned;          // [0] nnz readback, [1..] scratch
  Ctl* h_ctl;                  // pinned mirror of ctl
  DevVec<MonoDesc> descs;
  DevVec<BsGroup> grp_ops;     // grouped bit-sliced ops of the current call (LDS-plane kernel)
  std::vector<BsGroup> h_grp;
  DevVec<RpRec> rp_prog;       // register-plane programs of the current call
  std::vector<RpRec> h_rp;     // the program of the run being prepared
  std::vector<RpRec> h_rp_call; // sim_apply_gates_static: the programs uploaded since the last drain
  std::vector<sim_gate> conv;  // sim_apply_ops: converted ops, kept between calls
  RunCompiler rc;              // MONO descriptors and bytecode of the current call
  DevVec<MeasRec> recs;
  DevVec<int32_t> outcomes;
  // host knowledge of the entry count
  bool nnz_known;
  uint64_t nnz_exact, nnz_ub;
  uint64_t last_updates, last_pruned;
  uint64_t last_ix[4];
  double last_mass;
};

namespace {

int block_of(const sim_t* s) { return s->cfg.block ? (int)s->cfg.block : 256; }

// Profiler: bracket a launch with two events from the pool.
hipEvent_t next_event(sim_t* s) {
  if (s->ev_used == s->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->ev_pool.push_back(e);
  }
  return s->ev_pool[s->ev_used++];
}

// Wall-clock timer of a host class.
struct HTimer {
  sim_t* s;
  int cls;
  std::chrono::steady_clock::time_point t0;
  HTimer(sim_t* s_, int c) : s(s_), cls(c), t0(std::chrono::steady_clock::now()) {}
  ~HTimer() {
    s->k_launches[cls]++;
    s->k_ms[cls] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

hipError_t timed_sync(sim_t* s) {
  HTimer t_(s, KC_H_SYNC);
  return hipStreamSynchronize(s->stream);
}

struct KTimer {
  sim_t* s;
  int cls;
  size_t idx = 0;
  bool on = false;
  KTimer(sim_t* s_, int c) : s(s_), cls(c) {
    s->k_launches[c]++;
    if (!((s->profile >> c) & 1u) || s->no_alloc) return;
    idx = s->ev_used;
    hipEvent_t e = next_event(s);
    on = e && hipEventRecord(e, s->stream) == hipSuccess;
  }
  ~KTimer() {
    if (!on) return;
    hipEvent_t e = next_event(s);
    if (e && hipEventRecord(e, s->stream) == hipSuccess) s->ev_pending.emplace_back(cls, idx);
  }
};

// After a stream synchronisation: fold pending event pairs into the totals.
void resolve_events(sim_t* s) {
  for (const auto& p : s->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev_pool[p.second], s->ev_pool[p.second + 1]) == hipSuccess)
      s->k_ms[p.first] += ms;
  }
  s->ev_pending.clear();
  s->ev_used = 0;
}

int mono_grid(const sim_t* s, uint64_t n) {
  const uint64_t per = (uint64_t)block_of(s) * 4;
  const uint64_t g = (n + per - 1) / per;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 2048));
}

int chunk_grid(uint64_t n) {
  const uint64_t g = (n + kTwoPassChunk - 1) / kTwoPassChunk;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, kMaxBlocks));
}

int flat_grid(uint64_t n) {
  const uint64_t g = (n + 255) / 256;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(g, 4096));
}

uint64_t* d_nnz(sim_t* s, int b) { return &s->ctl->nnz[b]; }

int read_nnz(sim_t* s, uint64_t* out) {
  HIP_TRY(hipMemcpyAsync(s->h_pinned, d_nnz(s, s->cur), 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(timed_sync(s));
  resolve_events(s);
  *out = s->h_pinned[0];
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = *out;
  return SIM_OK;
}

bool key_in_range(const sim_t* s, uint64_t lo, uint64_t hi) { return key_fits(s->cfg.n_qubits, lo, hi); }

int validate(const sim_t* s, const sim_gate& g, size_t i) {
  std::string why;
  if (gate_valid(s->cfg.n_qubits, g, &why)) return SIM_OK;
  return fail(SIM_E_ARG, "op " + std::to_string(i) + ": " + why);
}

// One 2048-entry tile per block: the hardware balances the tiles over the CUs.
int bs_grid(const sim_t* s, uint64_t n) {
  (void)s;
  const uint64_t tiles = (n + 2047) / 2048;
  return (int)std::max<uint64_t>(1, std::min<uint64_t>(tiles, 1u << 30));
}

// Branching op: index, count, scan, (capacity check), write, swap.
// split: the gate's partner mask touches a qubit that is the same in every
// entry, so no entry has a partner: no index is filled, built or probed, and
// the evaluation runs with no partner array.
int run_u2(sim_t* s, const sim_gate& g, bool* over, bool split) {
  *over = false;
  const uint64_t cap = s->cfg.capacity;
  uint64_t ub = s->nnz_known ? s->nnz_exact : s->nnz_ub;
  bool check = false;
  if (2 * ub > cap) {
    uint64_t n;
    int rc = read_nnz(s, &n);
    if (rc) return rc;
    ub = n;
    check = 2 * n > cap;
  }
  const double lf = lf_of(&s->cfg);
  const uint64_t slots = std::min<uint64_t>(table_slots(ub, lf), s->L.slots);
  const int other = s->cur ^ 1;
  const uint64_t* nnz_in = d_nnz(s, s->cur);
  const U2Desc d = u2_desc(g, s->cfg.eps);
  const int G = chunk_grid(ub);
  if (!check && !(s->cfg.flags & (SIM_FLAG_U2_TWO_PASS | SIM_FLAG_U2_GLOBAL_INDEX)) && ub <= kLdsU2Max) {
    // Small state (2 ub <= capacity): the whole gate in one block, its
    // partner index in LDS; the global index is not touched.
    {
      KTimer t_(s, KC_U2_LDS);
      launch_u2_lds(s->stream, s->wide, s->buf[s->cur], s->buf[other], nnz_in, d, s->ctl, d_nnz(s, other));
    }
    HIP_TRY(hipGetLastError());
    s->cur = other;
    s->nnz_known = false;
    s->nnz_ub = std::min<uint64_t>(2 * ub, cap);
    return SIM_OK;
  }
  const uint64_t prior = s->table_dirty;
  const uint32_t* partner = split ? nullptr : s->partner;
  if (!split) {
    if (const uint64_t dirty = std::min<uint64_t>(prior, slots)) {
      KTimer t_(s, KC_FILL);
      launch_fill(s->stream, s->table, kEmptySlot, dirty);
    }
    s->table_dirty = std::max<uint64_t>(prior, slots);   // the build below writes into [0, slots)
    {
      KTimer t_(s, KC_BUILD);
      launch_index_build(s->stream, s->wide, s->buf[s->cur], nnz_in, s->table, slots - 1, d, s->partner,
                         (s->cfg.flags & SIM_FLAG_COUNT_INDEX) ? s->ctl : nullptr,
                         flat_grid(ub), 256);
    }
    {
      KTimer t_(s, KC_U2_PROBE);
      launch_u2_probe(s->stream, s->wide, s->buf[s->cur], nnz_in, s->table, slots - 1, d, s->partner,
                      (s->cfg.flags & SIM_FLAG_COUNT_INDEX) ? s->ctl : nullptr, flat_grid(ub),
                      256);
    }
  }
  if (!check && !(s->cfg.flags & SIM_FLAG_U2_TWO_PASS) && ub <= (uint64_t)kMaxBlocks * kU2Tile) {
    // Outputs fit (2 ub <= capacity): evaluate, scan and write in one pass.
    const uint32_t tile = u2_tile_for(ub);
    const int T = (int)std::max<uint64_t>(1, (ub + tile - 1) / tile);
    if (++s->u2_epoch >= (1u << 30)) {   // epochs are 30 bits: start over on cleared words
      launch_fill(s->stream, s->status, 0ull, kMaxBlocks);
      s->u2_epoch = 1;
    }
    {
      KTimer t_(s, KC_U2_WRITE);
      launch_u2_fused(s->stream, s->wide, s->buf[s->cur], s->buf[other], nnz_in, partner, d, s->ctl, s->status,
                      s->ticket_base, s->u2_epoch, d_nnz(s, other), s->table, split ? 0 : slots, T, tile);
    }
    HIP_TRY(hipGetLastError());
    s->ticket_base += (uint32_t)T;   // only a launched kernel advances the device counter
    if (!split) s->table_dirty = prior > slots ? prior : 0;   // [0, slots) emptied by the kernel
    s->cur = other;
    s->nnz_known = false;
    s->nnz_ub = std::min<uint64_t>(2 * ub, cap);
    return SIM_OK;
  }
  {
    KTimer t_(s, KC_U2_COUNT);
    launch_u2_count(s->stream, s->wide, s->buf[s->cur], nnz_in, d, partner, s->bs.tot, s->ctl, G, 256);
  }
  {
    KTimer t_(s, KC_SCAN);
    launch_scan(s->stream, s->bs.tot, G, d_nnz(s, other), s->ctl, s->wide ? 32u : 24u, cap);
  }
  HIP_TRY(hipGetLastError());
  if (check) {
    HIP_TRY(hipMemcpyAsync(s->h_pinned, d_nnz(s, other), 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(timed_sync(s));
    if (s->h_pinned[0] > cap) {
      *over = true;
      return SIM_OK;
    }
  }
  {
    KTimer t_(s, KC_U2_WRITE);
    launch_u2_write(s->stream, s->wide, s->buf[s->cur], s->buf[other], nnz_in, partner, s->bs.tot, d, s->ctl, G, 256);
  }
  HIP_TRY(hipGetLastError());
  s->cur = other;
  s->nnz_known = false;
  s->nnz_ub = std::min<uint64_t>(2 * ub, cap);
  return SIM_OK;
}

// Measurement: reduce, decide, write.  A chain of consecutive measurements
// skips the reduce after the first: each write forms the sums of the next
// measured qubit over the entries it writes (q_next >= 0), and the next
// measurement takes block b's input range from the offsets that write used.
// s->mchain records such sums (their qubit, grid and offsets array).
int run_measure(sim_t* s, uint32_t q, double u, int32_t forced, MeasRec* rec, int32_t* outcome, bool* bad,
                int32_t q_next = -1) {
  *bad = false;
  const uint64_t ub = s->nnz_known ? s->nnz_exact : s->nnz_ub;
  // 8192 entries per block: a quarter of the partial sums the decide kernel
  // reads, each block still several tiles of work.
  const int G = (int)std::max<uint64_t>(1, std::min<uint64_t>((ub + kMeasChunk - 1) / kMeasChunk, kMaxBlocks));
  const int other = s->cur ^ 1;
  const uint64_t* nnz_in = d_nnz(s, s->cur);
  const bool chained = s->mchain.valid && s->mchain.q == q && s->mchain.grid == G;
  const uint32_t* in_off = chained ? s->mchain.off : nullptr;
  uint32_t* out_off = in_off == s->bs.tot ? s->bs.tot2 : s->bs.tot;
  s->mchain.valid = false;
  if (!chained) {
    KTimer t_(s, KC_M_REDUCE);
    launch_measure_reduce(s->stream, s->wide, s->buf[s->cur], nnz_in, q, s->bs, G, 256);
  }
  {
    KTimer t_(s, KC_M_DECIDE);
    launch_measure_decide(s->stream, s->bs.part, s->bs.cnt1, out_off, G, nnz_in, d_nnz(s, other), u, forced, rec,
                          outcome, s->ctl, s->wide ? 32u : 24u, in_off);
  }
  HIP_TRY(hipGetLastError());
  if (forced >= 0 || ub == 0) {
    // A forced outcome may have zero probability: decide before touching the state.
    HIP_TRY(hipMemcpyAsync(s->h_pinned + 1, &rec->outcome, 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(timed_sync(s));
    int32_t o;
    std::memcpy(&o, s->h_pinned + 1, 4);
    if (o < 0) {
      *bad = true;
      return SIM_OK;
    }
  }
  {
    KTimer t_(s, KC_M_WRITE);
    launch_measure_write(s->stream, s->wide, s->buf[s->cur], s->buf[other], nnz_in, q, rec, out_off, in_off, q_next,
                         s->bs.part, s->bs.cnt1, G);
  }
  HIP_TRY(hipGetLastError());
  s->cur = other;
  s->nnz_known = false;
  s->nnz_ub = ub;
  if (q_next >= 0) s->mchain = {true, (uint32_t)q_next, G, out_off};
  return SIM_OK;
}

int read_ctl(sim_t* s) {
  HIP_TRY(hipMemcpyAsync(s->h_ctl, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(timed_sync(s));
  resolve_events(s);
  return SIM_OK;
}

}  // namespace

extern "C" {

size_t sim_workspace_bytes(const sim_config* cfg) {
  std::string why;
  if (!config_ok(cfg, &why)) return 0;
  return layout_of(cfg).total;
}

int sim_create(const sim_config* cfg, void* stream, void* workspace, size_t ws_bytes, sim_t** out) {
  std::string why;
  if (!out) return fail(SIM_E_ARG, "null output handle");
  *out = nullptr;
  if (!config_ok(cfg, &why)) return fail(SIM_E_ARG, why);
  sim_t* s = new (std::nothrow) sim_t();
  if (!s) return fail(SIM_E_NOMEM, "host allocation failed");
  s->cfg = *cfg;
  if (!s->cfg.fuse_max) s->cfg.fuse_max = 65536;
  s->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  if (hipError_t e = mono_rp_init(); e != hipSuccess) {
    delete s;
    return fail(SIM_E_HIP, std::string("mono_rp_init: ") + hipGetErrorString(e));
  }
  s->wide = cfg->n_qubits > 64;
  s->L = layout_of(cfg);
  if (workspace) {
    if (ws_bytes < s->L.total) {
      delete s;
      return fail(SIM_E_NOMEM, "workspace smaller than sim_workspace_bytes()");
    }
    s->ws = static_cast<char*>(workspace);
    s->ws_owned = false;
  } else {
    if (hipMalloc(&s->ws, s->L.total) != hipSuccess) {
      delete s;
      return fail(SIM_E_NOMEM, "hipMalloc of the state workspace failed");
    }
    s->ws_owned = true;
  }
  for (int b = 0; b < 2; ++b) {
    s->buf[b].key_lo = reinterpret_cast<uint64_t*>(s->ws + s->L.buf_lo[b]);
    s->buf[b].key_hi = s->wide ? reinterpret_cast<uint64_t*>(s->ws + s->L.buf_hi[b]) : nullptr;
    s->buf[b].amp = reinterpret_cast<double2*>(s->ws + s->L.buf_amp[b]);
  }
  s->table = reinterpret_cast<uint64_t*>(s->ws + s->L.table);
  s->partner = reinterpret_cast<uint32_t*>(s->ws + s->L.partner);
  s->bs.tot = reinterpret_cast<uint32_t*>(s->ws + s->L.tot);
  s->bs.tot2 = reinterpret_cast<uint32_t*>(s->ws + s->L.tot2);
  s->bs.cnt1 = reinterpret_cast<uint32_t*>(s->ws + s->L.cnt1);
  s->bs.part = reinterpret_cast<double2*>(s->ws + s->L.part);
  s->ctl = reinterpret_cast<Ctl*>(s->ws + s->L.ctl);
  s->status = reinterpret_cast<uint64_t*>(s->ws + s->L.status);
  if (hipHostMalloc(&s->h_pinned, 64) != hipSuccess || hipHostMalloc(&s->h_ctl, sizeof(Ctl)) != hipSuccess) {
    sim_destroy(s);
    return fail(SIM_E_NOMEM, "pinned host allocation failed");
  }
  std::memset(s->h_ctl, 0, sizeof(Ctl));
  if (hipMemcpyAsync(s->ctl, s->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, s->stream) != hipSuccess) {
    sim_destroy(s);
    return fail(SIM_E_HIP, "initialising the control block failed");
  }
  s->cur = 0;
  launch_fill(s->stream, s->status, 0ull, kMaxBlocks);   // epoch 0: no launch has published yet
  launch_fill(s->stream, s->table, kEmptySlot, s->L.slots);
  launch_set_basis(s->stream, s->buf[0], d_nnz(s, 0), 0, 0);
  if (hipStreamSynchronize(s->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    sim_destroy(s);
    return fail(SIM_E_HIP, "initial state setup failed");
  }
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = 1;
  s->last_updates = s->last_pruned = 0;
  for (int k = 0; k < 4; ++k) s->last_ix[k] = 0;
  s->last_mass = 0.0;
  *out = s;
  return SIM_OK;
}

int sim_destroy(sim_t* s) {
  if (!s) return SIM_OK;
  if (s->stream || s->ws) (void)hipStreamSynchronize(s->stream);
  s->descs.release();
  s->grp_ops.release();
  s->rp_prog.release();
  s->recs.release();
  s->outcomes.release();
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  if (s->h_pinned) (void)hipHostFree(s->h_pinned);
  if (s->h_ctl) (void)hipHostFree(s->h_ctl);
  if (s->ws_owned && s->ws) (void)hipFree(s->ws);
  delete s;
  return SIM_OK;
}

int sim_set_basis(sim_t* s, sim_key k) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  if (!key_in_range(s, k.lo, k.hi)) return fail(SIM_E_ARG, "basis key has bits above n_qubits");
  launch_set_basis(s->stream, s->buf[s->cur], d_nnz(s, s->cur), k.lo, k.hi);
  HIP_TRY(hipGetLastError());
  HIP_TRY(timed_sync(s));
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = 1;
  s->uni_lo = s->uni_hi = ~0ull;
  return SIM_OK;
}

int sim_import_state(sim_t* s, const sim_key* keys, const sim_c64* amps, uint64_t n) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  if (n > s->cfg.capacity) return fail(SIM_E_CAPACITY, "import larger than capacity");
  if (n && (!keys || !amps)) return fail(SIM_E_ARG, "null import arrays");
  std::vector<uint64_t> lo(n), hi(n);
  for (uint64_t i = 0; i < n; ++i) {
    if (!key_in_range(s, keys[i].lo, keys[i].hi)) return fail(SIM_E_ARG, "import key has bits above n_qubits");
    lo[i] = keys[i].lo;
    hi[i] = keys[i].hi;
  }
  {
    std::vector<sim_key> sorted(keys, keys + n);
    std::sort(sorted.begin(), sorted.end(), [](const sim_key& a, const sim_key& b) {
      return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo;
    });
    for (uint64_t i = 1; i < n; ++i)
      if (sorted[i].lo == sorted[i - 1].lo && sorted[i].hi == sorted[i - 1].hi)
        return fail(SIM_E_ARG, "duplicate key in import");
  }
  HIP_TRY(timed_sync(s));
  const Buf& b = s->buf[s->cur];
  if (n) {
    HIP_TRY(hipMemcpy(b.key_lo, lo.data(), n * 8, hipMemcpyHostToDevice));
    if (s->wide) HIP_TRY(hipMemcpy(b.key_hi, hi.data(), n * 8, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b.amp, amps, n * 16, hipMemcpyHostToDevice));
  }
  s->h_pinned[2] = n;
  HIP_TRY(hipMemcpyAsync(d_nnz(s, s->cur), s->h_pinned + 2, 8, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(timed_sync(s));
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = n;
  uint64_t and_lo = ~0ull, and_hi = ~0ull, or_lo = 0, or_hi = 0;
  for (uint64_t i = 0; i < n; ++i) {
    and_lo &= lo[i];
    and_hi &= hi[i];
    or_lo |= lo[i];
    or_hi |= hi[i];
  }
  s->uni_lo = ~(and_lo ^ or_lo);   // bits equal in every imported label (all, for none)
  s->uni_hi = ~(and_hi ^ or_hi);
  return SIM_OK;
}

namespace {

// One standard-gate record as a sim_gate; false for an unknown kind.
bool convert_op(const sim_op& o, sim_gate& out) {
  const double h = M_SQRT1_2;
  sim_gate g;
  std::memset(&g, 0, sizeof g);
  g.target = o.target;
  g.ctrl.lo = o.ctrl_lo;
  g.ctrl.hi = o.ctrl_hi;
  g.cap = o.cap;
  g.forced = -1;
  for (int k = 0; k < 4; ++k) g.m[k] = sim_c64{0.0, 0.0};
  const double c2 = std::cos(0.5 * o.param), s2 = std::sin(0.5 * o.param);
  g.op = SIM_OP_MONO;
  g.m[0] = g.m[1] = sim_c64{1.0, 0.0};
  switch (o.kind) {
    case SIM_K_X: g.flip = 1; break;
    case SIM_K_Y: g.flip = 1; g.m[0] = sim_c64{0.0, 1.0}; g.m[1] = sim_c64{0.0, -1.0}; break;
    case SIM_K_Z: g.m[1] = sim_c64{-1.0, 0.0}; break;
    case SIM_K_S: g.m[1] = sim_c64{0.0, 1.0}; break;
    case SIM_K_SDG: g.m[1] = sim_c64{0.0, -1.0}; break;
    case SIM_K_T: g.m[1] = sim_c64{h, h}; break;
    case SIM_K_TDG: g.m[1] = sim_c64{h, -h}; break;
    case SIM_K_RZ: g.m[0] = sim_c64{c2, -s2}; g.m[1] = sim_c64{c2, s2}; break;
    case SIM_K_PHASE: g.m[1] = sim_c64{std::cos(o.param), std::sin(o.param)}; break;
    case SIM_K_H:
      g.op = SIM_OP_U2;
      g.m[0] = sim_c64{h, 0.0}; g.m[1] = sim_c64{h, 0.0}; g.m[2] = sim_c64{h, 0.0}; g.m[3] = sim_c64{-h, 0.0};
      break;
    case SIM_K_RX:
      g.op = SIM_OP_U2;
      g.m[0] = sim_c64{c2, 0.0}; g.m[1] = sim_c64{0.0, -s2}; g.m[2] = sim_c64{0.0, -s2}; g.m[3] = sim_c64{c2, 0.0};
      break;
    case SIM_K_RY:
      g.op = SIM_OP_U2;
      g.m[0] = sim_c64{c2, 0.0}; g.m[1] = sim_c64{-s2, 0.0}; g.m[2] = sim_c64{s2, 0.0}; g.m[3] = sim_c64{c2, 0.0};
      break;
    case SIM_K_MEASURE:
      g.op = SIM_OP_MEASURE;
      g.m[0] = g.m[1] = sim_c64{0.0, 0.0};
      g.u = o.param;
      g.forced = o.forced;
      g.cap = 0;
      break;
    default:
      return false;
  }
  out = g;
  return true;
}

}  // namespace

int sim_gates_from_ops(const sim_op* ops, size_t n, sim_gate* out) {
  if (n && (!ops || !out)) return fail(SIM_E_ARG, "null op arrays");
  std::vector<size_t> bad(HostPool::kMaxThreads, SIZE_MAX);
  parallel_parts(n, 16384, [&](size_t b, size_t e, size_t p) {
    for (size_t i = b; i < e; ++i)
      if (!convert_op(ops[i], out[i])) {
        bad[p] = i;
        return;
      }
  });
  const size_t i = *std::min_element(bad.begin(), bad.end());
  if (i != SIZE_MAX) {
    char msg[96];
    snprintf(msg, sizeof msg, "op %zu: unknown gate kind %u", i, ops[i].kind);
    return fail(SIM_E_ARG, msg);
  }
  return SIM_OK;
}

}  // extern "C"

namespace {

// ---- allocation-free variant: device buffers of a call in static memory ----
// Gates per sim_apply_gates_static call, and the static scratch behind it:
// descriptors of the per-entry fused pass, measurement records and outcomes,
// then register-plane programs (a ring, as in the allocating form).
constexpr size_t kStaticMaxGates = 65536;
constexpr size_t kStaticDescBytes = kStaticMaxGates * sizeof(MonoDesc);
constexpr size_t kStaticRecBytes = kStaticMaxGates * sizeof(MeasRec);
constexpr size_t kStaticOutBytes = kStaticMaxGates * sizeof(int32_t);
constexpr size_t kStaticScratchBytes = 32u << 20;
static_assert(kStaticDescBytes + kStaticRecBytes + kStaticOutBytes < kStaticScratchBytes / 2, "scratch layout");
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                  // guards g_scratch_ptr
char* g_scratch_ptr[kMaxDevices] = {};    // device address of `scratch`, per device
std::mutex g_static_call_mu[kMaxDevices]; // one allocation-free call per device at a time

// The address of this device's copy of `scratch`, looked up once per device
// with that device current.
int static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SIM_E_ARG, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev) HIP_TRY(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(SIM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return SIM_OK;
}

// Device buffers of one apply call.
struct CallBufs {
  bool fixed = false;          // carved from the static scratch (no growth; uploads from pageable memory)
  MonoDesc* descs = nullptr;
  MeasRec* recs = nullptr;
  int32_t* outcomes = nullptr;
  RpRec* rp = nullptr;         // fixed: the program ring
  size_t rp_cap = 0;           // records
};

int apply_impl(sim_t* s, const sim_gate* gates, size_t n, int32_t* outcomes, sim_stats* stats, CallBufs cb) {
  s->mchain.valid = false;
  sim_stats st;
  std::memset(&st, 0, sizeof st);
  size_t n_mono = 0, n_meas = 0;
  const bool bs_allowed = s->cfg.mono_mode != SIM_MONO_DIRECT;
  {
    HTimer t_(s, KC_H_PREPARE);
    // Validate everything first (an invalid op applies nothing), count the
    // classes and build the phase/permutation descriptors, on the host pool.
    std::vector<size_t> bad(HostPool::kMaxThreads, SIZE_MAX), pm(HostPool::kMaxThreads + 1, 0),
        pmeas(HostPool::kMaxThreads, 0);
    parallel_parts(n, 16384, [&](size_t b, size_t e, size_t p) {
      std::string why;
      size_t mono = 0, meas = 0;   // counted locally: the shared arrays are written once per part
      for (size_t i = b; i < e; ++i) {
        if (!gate_valid(s->cfg.n_qubits, gates[i], &why)) {
          bad[p] = i;
          return;
        }
        mono += gates[i].op == SIM_OP_MONO;
        meas += gates[i].op == SIM_OP_MEASURE;
      }
      pm[p + 1] = mono;
      pmeas[p] = meas;
    });
    const size_t first_bad = *std::min_element(bad.begin(), bad.end());
    if (first_bad != SIZE_MAX) return validate(s, gates[first_bad], first_bad);
    for (size_t p = 0; p < HostPool::kMaxThreads; ++p) {
      pm[p + 1] += pm[p];
      n_meas += pmeas[p];
    }
    n_mono = pm[HostPool::kMaxThreads];
    s->rc.descs.resize(n_mono);
    parallel_parts(n, 16384, [&](size_t b, size_t e, size_t p) {
      for (size_t i = b, k = pm[p]; i < e; ++i)
        if (gates[i].op == SIM_OP_MONO) s->rc.descs[k++] = mono_desc(gates[i]);
    });
  }
  // Bit-sliced bytecode of every phase/permutation op (used by eligible
  // runs), compiled on a host thread while the first ops run; joined before
  // the first run needs it (and on every way out of this call).
  struct Joiner {
    std::thread t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } compiler;
  // (Small lists compile on this thread: starting a thread costs more.  The
  // allocation-free form starts no thread.)
  if (bs_allowed && (n_mono < 8192 || cb.fixed)) s->rc.compile(s->cfg.n_qubits);
  else if (bs_allowed) compiler.t = std::thread([s]() { s->rc.compile(s->cfg.n_qubits); });
  if (!cb.fixed) {
    HIP_TRY(s->descs.reserve(n_mono));
    HIP_TRY(s->recs.reserve(n_meas));
    HIP_TRY(s->outcomes.reserve(n_meas));
    cb.descs = s->descs.p;
    cb.recs = s->recs.p;
    cb.outcomes = s->outcomes.p;
  }
  // Descriptors are uploaded for the runs that take the per-entry kernel,
  // a window of runs at a time, and the bit-sliced groups run by run, both
  // from pinned staging (asynchronous).
  Staging<MonoDesc> h_desc(s->stream);
  Staging<BsGroup> h_grp_pin(s->stream);
  // Register-plane programs go through pinned staging into rp_prog at
  // rp_used; when a run's program does not fit, the stream is drained (every
  // earlier program has been read) and filling starts over at 0.
  Staging<RpRec> h_rp_pin(s->stream);
  size_t rp_used = 0;
  const bool use_rp = !(s->cfg.flags & SIM_FLAG_BS_LDS);
  size_t desc_lo = 0, desc_hi = 0;   // descriptors [desc_lo, desc_hi) are on the device
  // Grouped kernel ops of the bit-sliced runs, appended run by run.  A run
  // of k > 0 ops has at most k + 1 groups (every group but an evening pad
  // holds an op), so reserving two groups per op before the first run keeps
  // the host copies of in-flight uploads in place.
  s->h_grp.clear();
  bool compiled = !bs_allowed;
  auto ensure_compiled = [&]() -> int {
    if (compiled) return SIM_OK;
    {
      HTimer t_(s, KC_H_PREPARE);
      if (compiler.t.joinable()) compiler.t.join();
    }
    compiled = true;
    if (use_rp && cb.fixed) {
      s->h_rp_call.clear();
      s->h_rp_call.reserve(std::min(cb.rp_cap, 4 * s->rc.ops.size() + 64));
    } else if (use_rp) {
      HIP_TRY(s->rp_prog.reserve(4 * s->rc.ops.size() + 64));
      HIP_TRY(h_rp_pin.reserve(4 * s->rc.ops.size() + 64));
      cb.rp = s->rp_prog.p;
      cb.rp_cap = s->rp_prog.n;
    } else {
      s->h_grp.reserve(2 * s->rc.ops.size() + 2);
      HIP_TRY(s->grp_ops.reserve(2 * s->rc.ops.size() + 2));
      HIP_TRY(h_grp_pin.reserve(2 * s->rc.ops.size() + 2));
    }
    return SIM_OK;
  };

  // Speculative grouping.  Before the host blocks to read an entry count
  // for a cap decision (the GPU drains meanwhile), a helper thread groups the
  // run that follows if this and every later capped branching gate up to the
  // next stop are skipped -- the usual case once the state sits at its cap.
  // When the run then ends exactly there, its groups are ready and the GPU
  // does not wait for the host to group it; otherwise they are dropped.
  struct Spec {
    std::thread t;
    bool ready = false;          // t has run (or runs) for [begin, begin + len)
    size_t begin = 0, len = 0;
    std::vector<BsGroup> grp;
    std::vector<RpRec> rp;       // register-plane program (use_rp)
    BsRun delta{};               // run constants the grouping moved (see RunCompiler::group)
    void join() {
      if (t.joinable()) t.join();
    }
    ~Spec() { join(); }
  } spec;

  int result = SIM_OK;
  size_t run_begin = 0, run_len = 0, mono_seen = 0, meas_seen = 0;
  auto flush = [&]() -> int {
    if (!run_len) return SIM_OK;
    const uint64_t ub = s->nnz_known ? s->nnz_exact : s->nnz_ub;
    uint32_t run_flags = 0;
    for (size_t k = run_begin; k < run_begin + run_len; ++k) {
      if (s->rc.descs[k].flags & kHasPhase) run_flags |= kRunPhase;
      if (s->rc.descs[k].flags & kFlip) run_flags |= kRunFlip;
    }
    // Algorithmic bytes per entry: label read (+ write if a gate flips),
    // amplitude read and write if a gate has a phase.
    const uint32_t kb = s->wide ? 16u : 8u;
    const uint32_t run_bpe = kb + ((run_flags & kRunFlip) ? kb : 0u) + ((run_flags & kRunPhase) ? 32u : 0u);
    BsRun br;
    if (bs_allowed) {
      int rc = ensure_compiled();
      if (rc) return rc;
    }
    if (bs_allowed && use_rp && s->rc.run_params(run_begin, run_len, s->cfg.mono_mode, s->cfg.bs_min_gates, &br)) {
      br.bytes_per_entry = run_bpe;
      {
        HTimer tg_(s, KC_H_GROUP);
        if (spec.ready && spec.begin == run_begin && spec.len == run_len) {
          spec.join();
          s->h_rp.swap(spec.rp);
          br.g_omega = (br.g_omega + spec.delta.g_omega) & 7u;
          br.g_turn += spec.delta.g_turn;
          spec.ready = false;
        } else {
          s->h_rp.clear();
          s->rc.schedule(run_begin, run_len, s->h_rp, &br);
        }
      }
      const size_t nr = s->h_rp.size();
      if (cb.fixed) {
        // Static ring: the host copy of each upload (pageable) stays in
        // h_rp_call until the stream has drained past it.
        if (nr > cb.rp_cap) return fail(SIM_E_NOMEM, "a run's program exceeds the static scratch (split the call)");
        if (rp_used + nr > cb.rp_cap || s->h_rp_call.size() + nr > s->h_rp_call.capacity()) {
          HIP_TRY(timed_sync(s));
          rp_used = 0;
          s->h_rp_call.clear();
          s->h_rp_call.reserve(std::min(cb.rp_cap, std::max<size_t>(2 * nr, 4096)));
        }
        const size_t h0 = s->h_rp_call.size();
        s->h_rp_call.insert(s->h_rp_call.end(), s->h_rp.begin(), s->h_rp.end());
        HIP_TRY(hipMemcpyAsync(cb.rp + rp_used, s->h_rp_call.data() + h0, nr * sizeof(RpRec), hipMemcpyHostToDevice,
                               s->stream));
      } else {
        if (rp_used + nr > s->rp_prog.n || (rp_used + nr) * sizeof(RpRec) > h_rp_pin.bytes) {
          HIP_TRY(timed_sync(s));
          rp_used = 0;
          HIP_TRY(s->rp_prog.reserve(2 * nr));
          HIP_TRY(h_rp_pin.reserve(2 * nr));
          cb.rp = s->rp_prog.p;
          cb.rp_cap = s->rp_prog.n;
        }
        std::memcpy(h_rp_pin.p + rp_used, s->h_rp.data(), nr * sizeof(RpRec));
        HIP_TRY(hipMemcpyAsync(cb.rp + rp_used, h_rp_pin.p + rp_used, nr * sizeof(RpRec), hipMemcpyHostToDevice,
                               s->stream));
      }
      {
        KTimer t_(s, KC_MONO);
        launch_mono_rp(s->stream, s->buf[s->cur], d_nnz(s, s->cur), cb.rp + rp_used, (uint32_t)nr, br, s->ctl,
                       bs_grid(s, ub));
      }
      rp_used += nr;
      st.bitslice_passes++;
    } else if (bs_allowed && s->rc.run_params(run_begin, run_len, s->cfg.mono_mode, s->cfg.bs_min_gates, &br)) {
      br.bytes_per_entry = run_bpe;
      const size_t g0 = s->h_grp.size();
      {
        HTimer tg_(s, KC_H_GROUP);
        if (spec.ready && spec.begin == run_begin && spec.len == run_len) {
          spec.join();
          s->h_grp.insert(s->h_grp.end(), spec.grp.begin(), spec.grp.end());
          br.g_omega = (br.g_omega + spec.delta.g_omega) & 7u;
          br.g_turn += spec.delta.g_turn;
          spec.ready = false;
        } else {
          s->rc.group(run_begin, run_len, s->h_grp, &br);
        }
      }
      const size_t ng = s->h_grp.size() - g0;
      if (s->h_grp.size() > s->grp_ops.n) return fail(SIM_E_STATE, "bit-sliced op groups exceed their buffer");
      if (ng) {
        std::memcpy(h_grp_pin.p + g0, s->h_grp.data() + g0, ng * sizeof(BsGroup));
        HIP_TRY(hipMemcpyAsync(s->grp_ops.p + g0, h_grp_pin.p + g0, ng * sizeof(BsGroup), hipMemcpyHostToDevice,
                               s->stream));
      }
      KTimer t_(s, KC_MONO);
      launch_mono_bs(s->stream, s->buf[s->cur], d_nnz(s, s->cur), s->grp_ops.p + g0, (uint32_t)ng, br, s->ctl,
                     bs_grid(s, ub));
      st.bitslice_passes++;
    } else {
      if (run_begin < desc_lo || run_begin + run_len > desc_hi) {
        // This run and those after it, up to 1024 descriptors, in one copy
        // (the allocation-free form copies from the compiled descriptors,
        // which stay in place until the call returns).
        desc_lo = run_begin;
        desc_hi = std::min(s->rc.descs.size(), run_begin + std::max<size_t>(run_len, 1024));
        const MonoDesc* src = s->rc.descs.data();
        if (!cb.fixed) {
          HIP_TRY(h_desc.reserve(s->rc.descs.size()));
          std::memcpy(h_desc.p + desc_lo, s->rc.descs.data() + desc_lo, (desc_hi - desc_lo) * sizeof(MonoDesc));
          src = h_desc.p;
        }
        HIP_TRY(hipMemcpyAsync(cb.descs + desc_lo, src + desc_lo, (desc_hi - desc_lo) * sizeof(MonoDesc),
                               hipMemcpyHostToDevice, s->stream));
      }
      KTimer t_(s, KC_MONO);
      launch_mono(s->stream, s->wide, s->buf[s->cur], d_nnz(s, s->cur), cb.descs + run_begin, (uint32_t)run_len,
                  run_flags, run_bpe, s->ctl, mono_grid(s, ub), block_of(s));
    }
    HIP_TRY(hipGetLastError());
    st.mono_passes++;
    run_begin += run_len;
    run_len = 0;
    return SIM_OK;
  };
  // Start the speculative grouping of the run that would follow a skip of
  // capped gate i (see Spec).
  auto speculate = [&](size_t i) -> int {
    if (!bs_allowed || cb.fixed) return SIM_OK;
    int rc = ensure_compiled();
    if (rc) return rc;
    const size_t begin = run_len ? run_begin : mono_seen;
    size_t len = run_len;
    for (size_t j = i + 1; j < n && len < s->cfg.fuse_max; ++j) {
      const sim_gate& h = gates[j];
      if (h.op == SIM_OP_MONO) ++len;
      else if (h.op != SIM_OP_U2 || !h.cap) break;
    }
    if (len < 1024) return SIM_OK;   // short runs group in microseconds
    BsRun probe;
    if (!s->rc.run_params(begin, len, s->cfg.mono_mode, s->cfg.bs_min_gates, &probe)) return SIM_OK;
    if (spec.ready && spec.begin == begin && spec.len == len) return SIM_OK;
    spec.join();
    spec.ready = true;
    spec.begin = begin;
    spec.len = len;
    spec.t = std::thread([s, &spec, use_rp]() {
      spec.grp.clear();
      spec.rp.clear();
      spec.delta = BsRun{};
      if (use_rp) s->rc.schedule(spec.begin, spec.len, spec.rp, &spec.delta);
      else s->rc.group(spec.begin, spec.len, spec.grp, &spec.delta);
    });
    return SIM_OK;
  };
  size_t i = 0;
  for (; i < n; ++i) {
    const sim_gate& g = gates[i];
    if (g.op == SIM_OP_MONO) {
      // A flip keeps its target uniform only if every control is uniform.
      if (g.flip) {
        uint64_t& tw = g.target < 64 ? s->uni_lo : s->uni_hi;
        const uint64_t tb = 1ull << (g.target & 63);
        if ((tw & tb) && ((g.ctrl.lo & ~s->uni_lo) | (g.ctrl.hi & ~s->uni_hi))) tw &= ~tb;
      }
      if (run_len == 0) run_begin = mono_seen;
      ++run_len;
      ++mono_seen;
      if (run_len >= s->cfg.fuse_max) {
        int rc = flush();
        if (rc) return rc;
      }
      continue;
    }
    if (g.op == SIM_OP_U2) {
      // Skipped iff 2 * nnz > cap.  The exact count is read back only when
      // the tracked upper bound cannot settle it.
      if (g.cap && 2 * (s->nnz_known ? s->nnz_exact : s->nnz_ub) > g.cap) {
        uint64_t nnz = s->nnz_exact;
        if (!s->nnz_known) {
          int rc = speculate(i);
          if (rc) return rc;
          rc = read_nnz(s, &nnz);
          if (rc) return rc;
          st.host_syncs++;
        }
        if (2 * nnz > g.cap) {
          st.u2_skipped++;
          continue;
        }
      }
      int rc = flush();
      if (rc) return rc;
      bool over = false;
      const bool was_known = s->nnz_known;
      // Partner mask x (a standard gate's is its target bit).
      uint64_t x_lo = g.x.lo, x_hi = g.x.hi;
      if (!x_lo && !x_hi) (g.target < 64 ? x_lo : x_hi) = 1ull << (g.target & 63);
      const bool split = !(s->cfg.flags & SIM_FLAG_NO_UNIFORM) && ((x_lo & s->uni_lo) | (x_hi & s->uni_hi));
      rc = run_u2(s, g, &over, split);
      if (rc) return rc;
      if (!was_known && s->nnz_known) st.host_syncs++;
      if (over) {
        result = fail(SIM_E_CAPACITY, "branching gate would exceed the state capacity");
        break;
      }
      s->uni_lo &= ~x_lo;
      s->uni_hi &= ~x_hi;
      st.u2_applied++;
      if (split) st.u2_split++;
      continue;
    }
    // measurement
    int rc = flush();
    if (rc) return rc;
    bool bad = false;
    // A measurement right after this one takes its sums from this write.
    const int32_t q_next = i + 1 < n && gates[i + 1].op == SIM_OP_MEASURE ? (int32_t)gates[i + 1].target : -1;
    rc = run_measure(s, g.target, g.u, g.forced, cb.recs + meas_seen, cb.outcomes + meas_seen, &bad, q_next);
    if (rc) return rc;
    if (bad) {
      result = fail(SIM_E_STATE, "measurement outcome has zero probability");
      break;
    }
    (g.target < 64 ? s->uni_lo : s->uni_hi) |= 1ull << (g.target & 63);
    st.measures++;
    ++meas_seen;
  }
  if (result == SIM_OK) {
    int rc = flush();
    if (rc) return rc;
  }
  if (outcomes && meas_seen)
    HIP_TRY(hipMemcpyAsync(outcomes, cb.outcomes, meas_seen * 4, hipMemcpyDeviceToHost, s->stream));
  int rc = read_ctl(s);
  if (rc) return rc;
  if (const uint32_t err = s->h_ctl->error) {
    // Cleared whatever the result (a forced zero-probability outcome sets it
    // too), so that it never carries over to a later call.
    s->h_ctl->error = 0;
    HIP_TRY(hipMemcpyAsync(&s->ctl->error, &s->h_ctl->error, 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(timed_sync(s));
    if (result == SIM_OK)
      result = (err & 2u)   ? fail(SIM_E_HIP, "single-pass branching kernel gave up waiting for a tile")
               : (err & 4u) ? fail(SIM_E_HIP, "one-block branching kernel launched on a state too large for it")
                                      : fail(SIM_E_STATE, "measurement of an empty state");
  }
  s->mchain.valid = false;
  st.gates_applied = i;
  st.updates = s->h_ctl->updates - s->last_updates;
  st.pruned = s->h_ctl->pruned - s->last_pruned;
  st.pruned_mass = s->h_ctl->pruned_mass - s->last_mass;
  st.index_inserts = s->h_ctl->ix[0] - s->last_ix[0];
  st.index_cas = s->h_ctl->ix[1] - s->last_ix[1];
  st.index_lookups = s->h_ctl->ix[2] - s->last_ix[2];
  st.index_probes = s->h_ctl->ix[3] - s->last_ix[3];
  for (int k = 0; k < 4; ++k) s->last_ix[k] = s->h_ctl->ix[k];
  st.peak_nnz = s->h_ctl->peak;
  s->last_updates = s->h_ctl->updates;
  s->last_pruned = s->h_ctl->pruned;
  s->last_mass = s->h_ctl->pruned_mass;
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = s->h_ctl->nnz[s->cur];
  if (s->nnz_exact > st.peak_nnz) st.peak_nnz = s->nnz_exact;
  if (stats) *stats = st;
  return result;
}

}  // namespace

extern "C" {

int sim_apply_gates(sim_t* s, const sim_gate* gates, size_t n, int32_t* outcomes, sim_stats* stats) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  if (n && !gates) return fail(SIM_E_ARG, "null gate array");
  return apply_impl(s, gates, n, outcomes, stats, CallBufs{});
}

int sim_apply_gates_static(sim_t* s, const sim_gate* gates, size_t n, int32_t* outcomes, sim_stats* stats) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  if (n && !gates) return fail(SIM_E_ARG, "null gate array");
  if (n > kStaticMaxGates)
    return fail(SIM_E_ARG, "sim_apply_gates_static takes at most " + std::to_string(kStaticMaxGates) + " ops per call");
  if (s->cfg.flags & SIM_FLAG_BS_LDS) return fail(SIM_E_ARG, "sim_apply_gates_static does not run the LDS-plane pass");
  char* base = nullptr;
  int rc = static_scratch(s->device, &base);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_static_call_mu[s->device]);
  CallBufs cb;
  cb.fixed = true;
  cb.descs = reinterpret_cast<MonoDesc*>(base);
  cb.recs = reinterpret_cast<MeasRec*>(base + kStaticDescBytes);
  cb.outcomes = reinterpret_cast<int32_t*>(base + kStaticDescBytes + kStaticRecBytes);
  const size_t rp_off = (kStaticDescBytes + kStaticRecBytes + kStaticOutBytes + 255) / 256 * 256;
  cb.rp = reinterpret_cast<RpRec*>(base + rp_off);
  cb.rp_cap = (kStaticScratchBytes - rp_off) / sizeof(RpRec);
  s->no_alloc = true;
  rc = apply_impl(s, gates, n, outcomes, stats, cb);
  s->no_alloc = false;
  return rc;
}

int sim_apply_ops(sim_t* s, const sim_op* ops, size_t n, int32_t* outcomes, sim_stats* stats) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  // The conversion buffer stays with the handle, so repeated calls reuse
  // memory that is already mapped.
  try {
    if (s->conv.size() < n) s->conv.resize(n);
  } catch (const std::bad_alloc&) {
    return fail(SIM_E_NOMEM, "host allocation of the converted ops failed");
  }
  int rc = sim_gates_from_ops(ops, n, s->conv.data());
  if (rc) return rc;
  return sim_apply_gates(s, s->conv.data(), n, outcomes, stats);
}

int sim_apply_pauli(sim_t* s, const sim_pauli* terms, size_t n, sim_stats* stats) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  if (n && !terms) return fail(SIM_E_ARG, "null term array");
  std::vector<sim_gate> g(pauli_op_count(terms, n));
  size_t total = 0;
  int rc = sim_gates_from_pauli(terms, n, s->cfg.n_qubits, g.data(), g.size(), &total);
  if (rc) return rc;
  return sim_apply_gates(s, g.data(), total, nullptr, stats);
}

int sim_measure(sim_t* s, uint32_t qubit, double u, int32_t forced, int32_t* outcome, double* p1) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  sim_gate g;
  std::memset(&g, 0, sizeof g);
  g.op = SIM_OP_MEASURE;
  g.target = qubit;
  g.u = u;
  g.forced = forced;
  int rc = validate(s, g, 0);
  if (rc) return rc;
  HIP_TRY(s->recs.reserve(1));
  HIP_TRY(s->outcomes.reserve(1));
  bool bad = false;
  s->mchain.valid = false;
  rc = run_measure(s, qubit, u, forced, s->recs.p, s->outcomes.p, &bad);
  if (rc) return rc;
  MeasRec rec;
  HIP_TRY(hipMemcpyAsync(s->h_pinned + 4, s->recs.p, sizeof(MeasRec), hipMemcpyDeviceToHost, s->stream));
  rc = read_ctl(s);
  if (rc) return rc;
  std::memcpy(&rec, s->h_pinned + 4, sizeof rec);
  s->nnz_known = true;
  s->nnz_exact = s->nnz_ub = s->h_ctl->nnz[s->cur];
  if (bad || rec.outcome < 0) {
    if (s->h_ctl->error) {
      s->h_ctl->error = 0;
      HIP_TRY(hipMemcpyAsync(&s->ctl->error, &s->h_ctl->error, 4, hipMemcpyHostToDevice, s->stream));
      HIP_TRY(timed_sync(s));
    }
    return fail(SIM_E_STATE, "measurement outcome has zero probability or the state is empty");
  }
  if (outcome) *outcome = rec.outcome;
  if (p1) *p1 = rec.p1 / (rec.p0 + rec.p1);
  (qubit < 64 ? s->uni_lo : s->uni_hi) |= 1ull << (qubit & 63);   // collapsed: the bit is the outcome everywhere
  return SIM_OK;
}

int sim_nnz(sim_t* s, uint64_t* nnz) {
  if (!s || !nnz) return fail(SIM_E_ARG, "null argument");
  return read_nnz(s, nnz);
}

int sim_sync(sim_t* s) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  HIP_TRY(timed_sync(s));
  return SIM_OK;
}

int sim_export_state(sim_t* s, sim_key* keys, sim_c64* amps, uint64_t cap, uint64_t* nnz) {
  if (!s || !nnz) return fail(SIM_E_ARG, "null argument");
  uint64_t n;
  int rc = read_nnz(s, &n);
  if (rc) return rc;
  *nnz = n;
  if (cap < n) return fail(SIM_E_BUFFER, "export buffer smaller than nnz");
  if (!n) return SIM_OK;
  if (!keys || !amps) return fail(SIM_E_ARG, "null export arrays");
  const Buf& b = s->buf[s->cur];
  HIP_TRY(copy_state_to_host(b.key_lo, s->wide ? b.key_hi : nullptr, b.amp, n, keys, amps));
  return SIM_OK;
}

int sim_export_state_soa(sim_t* s, uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps, uint64_t cap, uint64_t* nnz) {
  if (!s || !nnz) return fail(SIM_E_ARG, "null argument");
  uint64_t n;
  int rc = read_nnz(s, &n);
  if (rc) return rc;
  *nnz = n;
  if (cap < n) return fail(SIM_E_BUFFER, "export buffer smaller than nnz");
  if (!n) return SIM_OK;
  if (!key_lo || !amps) return fail(SIM_E_ARG, "null export arrays");
  const Buf& b = s->buf[s->cur];
  HIP_TRY(copy_state_to_host_soa(b.key_lo, s->wide ? b.key_hi : nullptr, b.amp, n, key_lo, key_hi, amps));
  return SIM_OK;
}

int sim_device_state(sim_t* s, uint64_t** key_lo, uint64_t** key_hi, double** amp, uint64_t** dn) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  const Buf& b = s->buf[s->cur];
  if (key_lo) *key_lo = b.key_lo;
  if (key_hi) *key_hi = b.key_hi;
  if (amp) *amp = reinterpret_cast<double*>(b.amp);
  if (dn) *dn = d_nnz(s, s->cur);
  return SIM_OK;
}

int sim_set_tuning(sim_t* s, const sim_config* t) {
  if (!s || !t) return fail(SIM_E_ARG, "null argument");
  if (t->block != 0 && t->block != 64 && t->block != 128 && t->block != 256)
    return fail(SIM_E_ARG, "block must be 64, 128 or 256");
  if (t->mono_mode > SIM_MONO_BITSLICE) return fail(SIM_E_ARG, "unknown mono_mode");
  // The fused-pass kernel (SIM_FLAG_BS_LDS) is chosen at creation only.
  if (t->flags & SIM_FLAG_BS_LDS) return fail(SIM_E_ARG, "SIM_FLAG_BS_LDS is set at creation (sim_create) only");
  if (t->flags & ~(SIM_FLAG_U2_TWO_PASS | SIM_FLAG_U2_GLOBAL_INDEX | SIM_FLAG_COUNT_INDEX | SIM_FLAG_NO_UNIFORM))
    return fail(SIM_E_ARG, "unknown flags");
  if (t->load_factor != 0.0 && !(t->load_factor > 0.0 && t->load_factor <= 0.9))
    return fail(SIM_E_ARG, "load_factor must be in (0, 0.9]");
  s->cfg.fuse_max = t->fuse_max ? t->fuse_max : 65536;
  s->cfg.block = t->block;
  s->cfg.mono_mode = t->mono_mode;
  s->cfg.bs_min_gates = t->bs_min_gates;
  s->cfg.flags = (s->cfg.flags & SIM_FLAG_BS_LDS) | t->flags;
  if (t->load_factor >= lf_of(&s->cfg)) s->cfg.load_factor = t->load_factor;
  return SIM_OK;
}

int sim_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16) return fail(SIM_E_ARG, "sim_device_copy needs device pointers and a multiple of 16 bytes");
  launch_copy16(static_cast<hipStream_t>(stream), dst, src, bytes / 16);
  HIP_TRY(hipGetLastError());
  return SIM_OK;
}

int sim_set_profiling(sim_t* s, int on) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  HIP_TRY(timed_sync(s));
  resolve_events(s);
  if (on < 0 || on > SIM_PROFILE_MONO) return fail(SIM_E_ARG, "profiling mode must be 0, 1 or 2");
  s->profile = on == SIM_PROFILE_ALL ? (1u << KC_KERNELS) - 1u : on == SIM_PROFILE_MONO ? 1u << KC_MONO : 0u;
  return SIM_OK;
}

int sim_kernel_stats(sim_t* s, sim_kernel_stat* out, int cap, int* n) {
  if (!s || !n) return fail(SIM_E_ARG, "null argument");
  int rc = read_ctl(s);
  if (rc) return rc;
  *n = KC_COUNT;
  for (int c = 0; c < KC_COUNT && c < cap; ++c) {
    sim_kernel_stat& k = out[c];
    std::memset(&k, 0, sizeof k);
    std::snprintf(k.name, sizeof k.name, "%s", kClassNames[c]);
    k.launches = s->k_launches[c];
    k.total_ms = s->k_ms[c];
    if (c == KC_MONO) {
      k.alg_bytes = (double)(s->h_ctl->mono_bytes - s->mono_bytes_base);
      k.updates = (double)(s->h_ctl->mono_updates - s->mono_updates);
    }
    const int pass = c == KC_U2_COUNT  ? 0
                     : c == KC_U2_WRITE ? 1
                     : c == KC_M_REDUCE ? 2
                     : c == KC_M_WRITE  ? 3
                     : c == KC_U2_LDS   ? 4
                                        : -1;
    if (pass >= 0) k.alg_bytes = (double)(s->h_ctl->pass_bytes[pass] - s->pass_bytes_base[pass]);
  }
  return SIM_OK;
}

int sim_kernel_stats_reset(sim_t* s) {
  if (!s) return fail(SIM_E_ARG, "null handle");
  int rc = read_ctl(s);
  if (rc) return rc;
  for (int c = 0; c < KC_COUNT; ++c) {
    s->k_launches[c] = 0;
    s->k_ms[c] = 0.0;
  }
  s->mono_bytes_base = s->h_ctl->mono_bytes;
  for (int k = 0; k < 5; ++k) s->pass_bytes_base[k] = s->h_ctl->pass_bytes[k];
  s->mono_updates = s->h_ctl->mono_updates;
  return SIM_OK;
}

const char* sim_strerror(int code) {
  switch (code) {
    case SIM_OK: return "ok";
    case SIM_E_ARG: return "invalid argument";
    case SIM_E_NOMEM: return "out of memory";
    case SIM_E_CAPACITY: return "state capacity exceeded";
    case SIM_E_BUFFER: return "buffer too small";
    case SIM_E_HIP: return "HIP runtime error";
    case SIM_E_STATE: return "invalid state for the operation";
    default: return "unknown error";
  }
}

const char* sim_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
