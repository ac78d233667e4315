// Sparse state-vector ORACLE -- test infrastructure only.
//
// A plain, slow, obviously correct CPU implementation of the sparse simulation
// method of Jaques & Haner, "Leveraging state sparsity for more efficient
// quantum simulations" (arXiv 2105.01533).  Only the test suite, the smoke
// check and the benchmark's CPU-baseline leg may load this library; the GPU
// library never does, and the two share no code.
//
// The state is the paper's Sec. 3 data structure: unordered (label, amplitude)
// pairs for the nonzero amplitudes, here std::unordered_map from a 128-bit
// label to a complex<double>.  Qubit q is bit q of the label (Sec. 2.1: i_k is
// the k-th bit of i); qubits 64..127 live in the high word.
//
// Operations (Sec. 3.1):
//   * phase/permutation gates (at most one nonzero per row and column):
//     G(a_b |b>) = f(b) a_b |g(b)>, applied by rebuilding the map;
//   * branching gates (two nonzeros per row): Eq. 2 on the pair (b, b') with
//     b' = b xor 2^t; at most one look-up of the partner per label, and when
//     both partners are present only the label whose target bit is 1 emits;
//   * measurement: Born rule (Sec. 2.1), projection onto the outcome and
//     renormalisation.
// Queued mode (Sec. 3.2) applies a maximal run of phase/permutation gates to
// each label in turn, composing f and g as in the paper, before inserting the
// result into the new map.  Gate-by-gate mode rebuilds the map after every
// gate.  The two must agree bit for bit.  With orc_set_threads > 1, a queue of
// more than 64 gates on more than 4096 entries is applied by several threads
// (Sec. 5), again bit for bit as the serial loop.
//
// Readings where the paper is silent (also listed in the design notes):
//   * prune T_eps after every applied branching gate: drop an entry iff
//     re*re + im*im < eps, and always drop exact zeros (the paper stores only
//     nonzero amplitudes).  Phase/permutation gates never prune.
//   * a branching gate with cap != 0 is skipped iff 2*nnz > cap.
//   * measurement: P0, P1 are sums of |a|^2 over labels with the qubit 0 / 1,
//     taken in ascending label order; outcome 0 iff u < P0/(P0+P1) (unless
//     forced); the kept amplitudes are scaled by 1/sqrt(P_outcome).
//   * complex products are (a.re*b.re - a.im*b.im, a.re*b.im + a.im*b.re),
//     evaluated as written with no fused multiply-add.
//
// Pauli exponentials exp(-i theta P), controlled or not (Sec. 3's intrinsic
// operations): orc_run_pauli, from the closed form cos(theta) I - i sin(theta) P;
// its readings are listed at that function.
//
// Gate commuting (Sec. 3.3, Fig. 1): orc_run_commuting keeps, per qubit,
// queues of H, Rx and Ry gates that are pending after the phase/permutation
// queue, and commutes each incoming gate through them where a simple relation
// holds; otherwise it executes the queues of the qubits involved.  Its
// readings are listed at that function.
//
// Built with g++ -O2 -ffp-contract=off.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

struct Label {
  uint64_t lo, hi;
  bool operator==(const Label& o) const { return lo == o.lo && hi == o.hi; }
  bool operator<(const Label& o) const { return hi != o.hi ? hi < o.hi : lo < o.lo; }
};

struct LabelHash {
  size_t operator()(const Label& k) const {
    uint64_t x = k.lo * 0x9E3779B97F4A7C15ull ^ (k.hi + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
    return static_cast<size_t>(x ^ (x >> 29));
  }
};

struct Amp {
  double re, im;
};

Amp mul(Amp a, Amp b) {
  Amp r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}

Amp add(Amp a, Amp b) { return Amp{a.re + b.re, a.im + b.im}; }

using State = std::unordered_map<Label, Amp, LabelHash>;

// Op record written by the workload generator (48 bytes, little endian).
struct OpRecord {
  uint32_t kind, target;
  uint64_t ctrl_lo, ctrl_hi;
  double param;
  uint64_t cap;
  int32_t forced;
  uint32_t pad;
};
static_assert(sizeof(OpRecord) == 48, "op record layout");

enum Kind : uint32_t {
  kX = 0, kY, kZ, kS, kSdg, kT, kTdg, kRz, kPhase,
  kH = 9, kRx, kRy,
  kMeasure = 12
};

bool is_monomial(uint32_t k) { return k <= kPhase; }
bool is_branching(uint32_t k) { return k >= kH && k <= kRy; }

// A phase/permutation gate as the pair (f, g) of Sec. 3.2:
//   f(b) = m[bit_t(b)] when the controls are set (and has_phase), else 1;
//   g(b) = b xor (flip ? 2^t : 0) when the controls are set, else b.
struct Monomial {
  Label ctrl;
  unsigned target;
  bool flip;
  bool has_phase;
  Amp m[2];
};

// Gate matrices from Sec. 2.1: H = sqrt(0.5)[[1,1],[1,-1]], S = diag(1,i),
// X, Y, Z, and R_P(theta) = exp(-i theta P / 2).  T = diag(1, e^{i pi/4}) and
// the adjoints are the textbook definitions.  A column of a permutation-type
// matrix is read off as "input bit v goes to output bit v xor flip with factor
// m[v]".
Monomial monomial_of(const OpRecord& op) {
  Monomial g;
  g.ctrl = Label{op.ctrl_lo, op.ctrl_hi};
  g.target = op.target;
  g.flip = false;
  g.has_phase = true;
  const double h = std::sqrt(0.5);
  const Amp one{1.0, 0.0};
  g.m[0] = one;
  g.m[1] = one;
  switch (op.kind) {
    case kX:  // [[0,1],[1,0]]: |0> -> |1>, |1> -> |0>
      g.flip = true;
      g.has_phase = false;
      break;
    case kY:  // [[0,-i],[i,0]]: |0> -> i|1>, |1> -> -i|0>
      g.flip = true;
      g.m[0] = Amp{0.0, 1.0};
      g.m[1] = Amp{0.0, -1.0};
      break;
    case kZ:
      g.m[1] = Amp{-1.0, 0.0};
      break;
    case kS:
      g.m[1] = Amp{0.0, 1.0};
      break;
    case kSdg:
      g.m[1] = Amp{0.0, -1.0};
      break;
    case kT:
      g.m[1] = Amp{h, h};
      break;
    case kTdg:
      g.m[1] = Amp{h, -h};
      break;
    case kRz: {  // exp(-i theta Z / 2) = diag(e^{-i theta/2}, e^{+i theta/2})
      const double c = std::cos(0.5 * op.param), s = std::sin(0.5 * op.param);
      g.m[0] = Amp{c, -s};
      g.m[1] = Amp{c, s};
      break;
    }
    case kPhase:  // diag(1, e^{i theta})
      g.m[1] = Amp{std::cos(op.param), std::sin(op.param)};
      break;
    default:
      break;
  }
  return g;
}

// Branching 2x2 matrix U (row-major): out0 = U00 a0 + U01 a1, out1 = U10 a0 + U11 a1.
void matrix_of(const OpRecord& op, Amp u[4]) {
  const double h = std::sqrt(0.5);
  const double c = std::cos(0.5 * op.param), s = std::sin(0.5 * op.param);
  switch (op.kind) {
    case kH:
      u[0] = Amp{h, 0.0};
      u[1] = Amp{h, 0.0};
      u[2] = Amp{h, 0.0};
      u[3] = Amp{-h, 0.0};
      break;
    case kRx:  // exp(-i theta X / 2) = [[c, -i s], [-i s, c]]
      u[0] = Amp{c, 0.0};
      u[1] = Amp{0.0, -s};
      u[2] = Amp{0.0, -s};
      u[3] = Amp{c, 0.0};
      break;
    case kRy:  // exp(-i theta Y / 2) = [[c, -s], [s, c]]
      u[0] = Amp{c, 0.0};
      u[1] = Amp{-s, 0.0};
      u[2] = Amp{s, 0.0};
      u[3] = Amp{c, 0.0};
      break;
    default:
      u[0] = u[1] = u[2] = u[3] = Amp{0.0, 0.0};
  }
}

bool bit_of(const Label& k, unsigned q) {
  return q < 64 ? ((k.lo >> q) & 1u) : ((k.hi >> (q - 64)) & 1u);
}

Label with_bit(Label k, unsigned q, bool v) {
  uint64_t& w = q < 64 ? k.lo : k.hi;
  const uint64_t m = 1ull << (q & 63);
  w = v ? (w | m) : (w & ~m);
  return k;
}

bool controls_set(const Label& k, const Label& c) {
  return (k.lo & c.lo) == c.lo && (k.hi & c.hi) == c.hi;
}

// (f, g) applied to one (label, amplitude) pair.
void apply_monomial(const Monomial& g, Label& k, Amp& a) {
  if (!controls_set(k, g.ctrl)) return;
  const bool v = bit_of(k, g.target);
  if (g.has_phase) a = mul(a, g.m[v ? 1 : 0]);
  if (g.flip) k = with_bit(k, g.target, !v);
}

struct Trace {           // per-op record returned to the caller
  uint64_t nnz_in;
  int32_t applied;       // 1 applied, 0 skipped
  int32_t outcome;       // MEASURE: outcome, else -1
  double p0, p1;         // MEASURE: unnormalised probabilities
};
static_assert(sizeof(Trace) == 32, "trace layout");

struct Totals {
  uint64_t updates;      // sum over applied gates of nnz at input
  uint64_t u2_applied, u2_skipped, measures, mono_gates;
  uint64_t peak_nnz, pruned;
  double pruned_mass;
  uint64_t parallel_runs;   // queues applied by several threads (Sec. 5)
  // Diagnostic (no effect on the state): the smallest | |a|^2 - eps | / eps
  // over every entry T_eps examined (eps > 0), i.e. how close a prune
  // decision came to flipping; +inf when none was examined.
  double min_margin;
};

struct Oracle {
  unsigned n_qubits;
  double eps;
  State psi;
  Totals tot;
  unsigned threads = 1;   // queue application (Sec. 5); 1 = serial
};

bool drop(const Amp& a, double eps) {
  return (a.re * a.re + a.im * a.im < eps) || (a.re == 0.0 && a.im == 0.0);
}

// T_eps on a whole new state (after a branching operation): drop the entries
// drop() names, count them and their mass, and note the decision margin.
void prune(Oracle& o, State& out) {
  for (auto it = out.begin(); it != out.end();) {
    const double m2 = it->second.re * it->second.re + it->second.im * it->second.im;
    if (o.eps > 0.0) o.tot.min_margin = std::min(o.tot.min_margin, std::fabs(m2 - o.eps) / o.eps);
    if (drop(it->second, o.eps)) {
      o.tot.pruned++;
      o.tot.pruned_mass += m2;
      it = out.erase(it);
    } else {
      ++it;
    }
  }
}

void note_peak(Oracle& o) {
  if (o.psi.size() > o.tot.peak_nnz) o.tot.peak_nnz = o.psi.size();
}

// Branching operation, Eq. 2, with the pair rule of Sec. 3.1.
void apply_branching(Oracle& o, const OpRecord& op) {
  Amp u[4];
  matrix_of(op, u);
  const Label ctrl{op.ctrl_lo, op.ctrl_hi};
  const unsigned t = op.target;
  State out;
  out.reserve(o.psi.size() * 2);
  const Amp zero{0.0, 0.0};
  for (const auto& kv : o.psi) {
    const Label& k = kv.first;
    if (!controls_set(k, ctrl)) {
      out.emplace(k, kv.second);
      continue;
    }
    const Label k0 = with_bit(k, t, false), k1 = with_bit(k, t, true);
    const bool v = bit_of(k, t);
    auto it_partner = o.psi.find(v ? k0 : k1);    // the one look-up
    const bool partner = it_partner != o.psi.end();
    if (!v && partner) continue;                   // the bit-1 label emits the pair
    const Amp a0 = v ? (partner ? it_partner->second : zero) : kv.second;
    const Amp a1 = v ? kv.second : zero;
    out.emplace(k0, add(mul(u[0], a0), mul(u[1], a1)));
    out.emplace(k1, add(mul(u[2], a0), mul(u[3], a1)));
  }
  prune(o, out);   // T_eps on the whole new state
  o.psi.swap(out);
}

// Sec. 5: a queue longer than 64 gates on a state of more than 4096 entries is
// processed by several threads.  Here each thread takes a contiguous range of
// the map's buckets (reading a map concurrently is safe), applies every queued
// gate to each of its labels and keeps the results in a list of its own; the
// lists are then inserted into the new map one after the other.  Labels are
// independent, so every (label, amplitude) is bitwise what the serial loop
// computes; only the map's internal order can differ, and nothing downstream
// depends on it (branching outputs are written once per label, two-term sums
// commute, measurement sums run in sorted label order).
constexpr size_t kParallelMinGates = 64, kParallelMinStates = 4096;

void apply_monomial_run_parallel(Oracle& o, const std::vector<Monomial>& run) {
  const size_t nb = o.psi.bucket_count();
  const unsigned nt = o.threads;
  std::vector<std::vector<std::pair<Label, Amp>>> part(nt);
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nt; ++t) {
    pool.emplace_back([&, t] {
      const size_t b0 = nb * t / nt, b1 = nb * (t + 1) / nt;
      auto& mine = part[t];
      for (size_t b = b0; b < b1; ++b)
        for (auto it = o.psi.begin(b); it != o.psi.end(b); ++it) {
          Label k = it->first;
          Amp a = it->second;
          for (const Monomial& g : run) apply_monomial(g, k, a);
          mine.emplace_back(k, a);
        }
    });
  }
  for (auto& th : pool) th.join();
  State out;
  out.reserve(o.psi.size());
  for (const auto& mine : part)
    for (const auto& e : mine) out.emplace(e.first, e.second);
  o.psi.swap(out);
}

// Apply a run of phase/permutation gates: per label, all gates in order,
// then one insertion into the new map (Sec. 3.2).
void apply_monomial_run(Oracle& o, const std::vector<Monomial>& run) {
  if (run.empty()) return;
  if (o.threads > 1 && run.size() > kParallelMinGates && o.psi.size() > kParallelMinStates) {
    apply_monomial_run_parallel(o, run);
    o.tot.parallel_runs++;
    return;
  }
  State out;
  out.reserve(o.psi.size());
  for (const auto& kv : o.psi) {
    Label k = kv.first;
    Amp a = kv.second;
    for (const Monomial& g : run) apply_monomial(g, k, a);
    out.emplace(k, a);
  }
  o.psi.swap(out);
}

std::vector<std::pair<Label, Amp>> sorted_entries(const State& s) {
  std::vector<std::pair<Label, Amp>> v(s.begin(), s.end());
  std::sort(v.begin(), v.end(),
            [](const std::pair<Label, Amp>& a, const std::pair<Label, Amp>& b) { return a.first < b.first; });
  return v;
}

void probabilities(const Oracle& o, unsigned q, double* p0, double* p1) {
  double s0 = 0.0, s1 = 0.0;
  for (const auto& e : sorted_entries(o.psi)) {
    const double p = e.second.re * e.second.re + e.second.im * e.second.im;
    if (bit_of(e.first, q)) s1 += p; else s0 += p;
  }
  *p0 = s0;
  *p1 = s1;
}

// Returns the outcome, or -1 if the chosen outcome has zero probability.
int measure(Oracle& o, unsigned q, double u, int forced, double* p0, double* p1) {
  probabilities(o, q, p0, p1);
  const double tot = *p0 + *p1;
  if (!(tot > 0.0)) return -1;
  int outcome = forced >= 0 ? forced : (u < *p0 / tot ? 0 : 1);
  const double po = outcome ? *p1 : *p0;
  if (!(po > 0.0)) return -1;
  const double scale = 1.0 / std::sqrt(po);
  State out;
  out.reserve(o.psi.size());
  for (const auto& kv : o.psi)
    if (bit_of(kv.first, q) == (outcome == 1)) out.emplace(kv.first, Amp{kv.second.re * scale, kv.second.im * scale});
  o.psi.swap(out);
  return outcome;
}

bool op_valid(const Oracle& o, const OpRecord& op) {
  if (op.target >= o.n_qubits) return false;
  if (op.kind > kMeasure) return false;
  if (bit_of(Label{op.ctrl_lo, op.ctrl_hi}, op.target)) return false;
  if (o.n_qubits < 128) {
    const Label lim = o.n_qubits >= 64 ? Label{~0ull, o.n_qubits == 64 ? 0ull : ((1ull << (o.n_qubits - 64)) - 1)}
                                       : Label{(1ull << o.n_qubits) - 1, 0ull};
    if ((op.ctrl_lo & ~lim.lo) || (op.ctrl_hi & ~lim.hi)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

// Error codes: 0 ok, -1 bad argument, -2 zero-probability measurement outcome.
void* orc_create(unsigned n_qubits, double eps) {
  if (n_qubits == 0 || n_qubits > 128) return nullptr;
  Oracle* o = new Oracle();
  o->n_qubits = n_qubits;
  o->eps = eps;
  o->psi.emplace(Label{0, 0}, Amp{1.0, 0.0});
  std::memset(&o->tot, 0, sizeof(o->tot));
  o->tot.peak_nnz = 1;
  o->tot.min_margin = std::numeric_limits<double>::infinity();
  return o;
}

void orc_destroy(void* h) { delete static_cast<Oracle*>(h); }

int orc_set_basis(void* h, uint64_t lo, uint64_t hi) {
  Oracle& o = *static_cast<Oracle*>(h);
  o.psi.clear();
  o.psi.emplace(Label{lo, hi}, Amp{1.0, 0.0});
  return 0;
}

// Replace the state by n (label, amplitude) pairs; amp is interleaved re,im.
int orc_import(void* h, const uint64_t* lo, const uint64_t* hi, const double* amp, uint64_t n) {
  Oracle& o = *static_cast<Oracle*>(h);
  State s;
  s.reserve(n);
  for (uint64_t i = 0; i < n; ++i)
    if (!s.emplace(Label{lo[i], hi[i]}, Amp{amp[2 * i], amp[2 * i + 1]}).second) return -1;
  o.psi.swap(s);
  note_peak(o);
  return 0;
}

uint64_t orc_nnz(void* h) { return static_cast<Oracle*>(h)->psi.size(); }

// Threads for queue application (Sec. 5); 0 = the hardware's count.  Returns
// the count in use.
unsigned orc_set_threads(void* h, unsigned n) {
  Oracle& o = *static_cast<Oracle*>(h);
  if (n == 0) n = std::max(1u, std::thread::hardware_concurrency());
  o.threads = n;
  return n;
}

// Run ops.  queued != 0 applies maximal runs of phase/permutation gates per
// label (skipped branching gates do not end a run: they leave nnz unchanged).
// trace (optional, n entries) and outcomes (optional, one per MEASURE) are
// filled in order.  Returns 0, -1 (invalid op at index *bad) or -2.
int orc_run(void* h, const OpRecord* ops, uint64_t n, int queued, Trace* trace, int32_t* outcomes,
            uint64_t* bad) {
  Oracle& o = *static_cast<Oracle*>(h);
  std::vector<Monomial> run;
  uint64_t n_meas = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const OpRecord& op = ops[i];
    if (!op_valid(o, op)) {
      apply_monomial_run(o, run);
      if (bad) *bad = i;
      return -1;
    }
    Trace tr{o.psi.size(), 1, -1, 0.0, 0.0};
    if (is_monomial(op.kind)) {
      o.tot.updates += o.psi.size();
      o.tot.mono_gates++;
      run.push_back(monomial_of(op));
      if (!queued) {
        apply_monomial_run(o, run);
        run.clear();
      }
    } else if (is_branching(op.kind)) {
      if (op.cap != 0 && 2 * o.psi.size() > op.cap) {
        tr.applied = 0;
        o.tot.u2_skipped++;
      } else {
        apply_monomial_run(o, run);
        run.clear();
        o.tot.updates += o.psi.size();
        o.tot.u2_applied++;
        apply_branching(o, op);
        note_peak(o);
      }
    } else {  // measurement flushes the queue
      apply_monomial_run(o, run);
      run.clear();
      o.tot.measures++;
      const int r = measure(o, op.target, op.param, op.forced, &tr.p0, &tr.p1);
      if (r < 0) {
        if (bad) *bad = i;
        return -2;
      }
      tr.outcome = r;
      if (outcomes) outcomes[n_meas] = r;
      n_meas++;
    }
    if (trace) trace[i] = tr;
  }
  apply_monomial_run(o, run);
  return 0;
}

// ---- gate commuting (Sec. 3.3) ------------------------------------------------
//
// Pending gates, in the order they act after the state: the phase/permutation
// queue Q, then on each qubit q an H (if h[q]), then Rx(rx[q]), then Ry(ry[q])
// (the figure's rows, applied bottom-up).  An incoming gate G is moved ahead of
// the pending gates of its qubits by these relations; where none applies, the
// gates pending on G's qubits are executed first (Q as a whole, then each such
// qubit's H, Rx, Ry), and G is then queued or applied.
//   * H on q:   H Ry(a) = Ry(-a) H, then H H = I (the H queue bit toggles);
//               an Rx pending on q has no such relation -> execute q first.
//   * Rx on q:  joins Rx(a): Rx(b) Rx(a) = Rx(a + b); an Ry pending on q sits
//               after it -> execute q first.
//   * Ry on q:  joins Ry(a): Ry(a + b).
//     A joined angle of exactly 0 leaves no gate.
//   * phase/permutation gate: on a qubit with H pending, an X or Z (possibly
//     controlled) whose target is that qubit becomes Z or X (X H = H Z and
//     Z H = H X); any other pending gate on one of its qubits -> execute them
//     first; the gate then joins Q.
//   * a branching gate with controls or a skip cap, and a measurement: execute
//     the gates pending on its qubits, then apply it (a measurement also needs
//     Q, which is executed with them).
//   * at the end everything pending is executed (qubits in ascending order).
// Every gate applied to the state is appended to `log` (when given), in order.
namespace {

struct Commuter {
  Oracle& o;
  std::vector<uint8_t> h, has_rx, has_ry;
  std::vector<double> rx, ry;
  std::vector<OpRecord> q;
  std::vector<OpRecord>* log;

  Commuter(Oracle& o_, std::vector<OpRecord>* log_)
      : o(o_), h(o_.n_qubits, 0), has_rx(o_.n_qubits, 0), has_ry(o_.n_qubits, 0), rx(o_.n_qubits, 0.0),
        ry(o_.n_qubits, 0.0), log(log_) {}

  static OpRecord single(uint32_t kind, unsigned t, double param) {
    OpRecord r{};
    r.kind = kind;
    r.target = t;
    r.param = param;
    r.forced = -1;
    return r;
  }
  void record(const OpRecord& r) {
    if (log) log->push_back(r);
  }
  void apply_u2(const OpRecord& r) {
    record(r);
    o.tot.updates += o.psi.size();
    o.tot.u2_applied++;
    apply_branching(o, r);
    note_peak(o);
  }
  void execute_q() {
    std::vector<Monomial> run;
    for (const OpRecord& r : q) {
      record(r);
      o.tot.updates += o.psi.size();
      o.tot.mono_gates++;
      run.push_back(monomial_of(r));
    }
    apply_monomial_run(o, run);
    q.clear();
  }
  bool pending(unsigned t) const { return h[t] || has_rx[t] || has_ry[t]; }
  // Execute Q and the gates pending on the qubits in `qs` (ascending).
  void execute(std::vector<unsigned> qs) {
    std::sort(qs.begin(), qs.end());
    qs.erase(std::unique(qs.begin(), qs.end()), qs.end());
    execute_q();
    for (unsigned t : qs) {
      if (h[t]) apply_u2(single(kH, t, 0.0));
      if (has_rx[t]) apply_u2(single(kRx, t, rx[t]));
      if (has_ry[t]) apply_u2(single(kRy, t, ry[t]));
      h[t] = has_rx[t] = has_ry[t] = 0;
      rx[t] = ry[t] = 0.0;
    }
  }
  static std::vector<unsigned> qubits_of(const OpRecord& r) {
    std::vector<unsigned> qs{r.target};
    for (unsigned c = 0; c < 128; ++c)
      if (bit_of(Label{r.ctrl_lo, r.ctrl_hi}, c)) qs.push_back(c);
    return qs;
  }
  void join(uint8_t& has, double& angle, double add) {
    const double a = has ? angle + add : add;
    has = a != 0.0;
    angle = has ? a : 0.0;
  }
};

}  // namespace

// Returns 0, -1 (invalid op at *bad) or -2 (measurement with no valid outcome
// at *bad).  n_log receives the number of applied gates (all of them are
// written when log_cap allows).
int orc_run_commuting(void* hnd, const OpRecord* ops, uint64_t n, OpRecord* log, uint64_t log_cap, uint64_t* n_log,
                      int32_t* outcomes, uint64_t* bad) {
  Oracle& o = *static_cast<Oracle*>(hnd);
  std::vector<OpRecord> applied;
  Commuter c(o, &applied);
  uint64_t n_meas = 0;
  int rc = 0;
  for (uint64_t i = 0; i < n && rc == 0; ++i) {
    const OpRecord& op = ops[i];
    if (!op_valid(o, op)) {
      c.execute({});
      if (bad) *bad = i;
      rc = -1;
      break;
    }
    const unsigned t = op.target;
    const bool plain = op.ctrl_lo == 0 && op.ctrl_hi == 0 && op.cap == 0;
    if (is_monomial(op.kind)) {
      const std::vector<unsigned> qs = Commuter::qubits_of(op);
      std::vector<unsigned> hard;
      for (unsigned qb : qs) {
        const bool swappable = qb == t && (op.kind == kX || op.kind == kZ) && !c.has_rx[qb] && !c.has_ry[qb];
        if (c.has_rx[qb] || c.has_ry[qb] || (c.h[qb] && !swappable)) hard.push_back(qb);
      }
      if (!hard.empty()) c.execute(hard);
      OpRecord g = op;
      if (c.h[t]) g.kind = op.kind == kX ? kZ : kX;   // X H = H Z, Z H = H X
      c.q.push_back(g);
    } else if (op.kind == kH && plain) {
      if (c.has_rx[t]) {
        c.execute({t});
        c.h[t] = 1;
      } else {
        if (c.has_ry[t]) c.ry[t] = -c.ry[t];
        c.h[t] ^= 1;
      }
    } else if (op.kind == kRx && plain) {
      if (c.has_ry[t]) c.execute({t});
      c.join(c.has_rx[t], c.rx[t], op.param);
    } else if (op.kind == kRy && plain) {
      c.join(c.has_ry[t], c.ry[t], op.param);
    } else if (is_branching(op.kind)) {
      // Sent to the state as is; a capped gate may then be skipped there.
      c.execute(Commuter::qubits_of(op));
      if (op.cap != 0 && 2 * o.psi.size() > op.cap) {
        c.record(op);
        o.tot.u2_skipped++;
      } else {
        c.apply_u2(op);
      }
    } else {  // measurement
      c.execute({t});
      c.record(op);
      o.tot.measures++;
      double p0, p1;
      const int r = measure(o, t, op.param, op.forced, &p0, &p1);
      if (r < 0) {
        if (bad) *bad = i;
        rc = -2;
        break;
      }
      if (outcomes) outcomes[n_meas] = r;
      n_meas++;
    }
  }
  if (rc == 0) {
    std::vector<unsigned> all;
    for (unsigned qb = 0; qb < o.n_qubits; ++qb)
      if (c.pending(qb)) all.push_back(qb);
    c.execute(all);
  }
  if (n_log) *n_log = applied.size();
  if (log)
    for (uint64_t k = 0; k < applied.size() && k < log_cap; ++k) log[k] = applied[k];
  return rc;
}

// ---- Pauli exponentials (Sec. 3: an intrinsic operation with at most two ----
// nonzeros per row) -------------------------------------------------------------
//
// exp(-i theta P) for a Pauli string P, optionally controlled.  P is given by
// two masks: P acts as X on the qubits in x only, Y on those in both x and z,
// Z on those in z only, and as the identity elsewhere.  Since P^2 = I the
// operator is cos(theta) I - i sin(theta) P, and P|b> = c(b)|b xor x> with c(b)
// the product of the single-qubit entries of Sec. 2.1's X, Y, Z in the column
// of b's bit.  The oracle applies exactly that: every label b (with the
// controls set) sends cos(theta) a_b to b and -i sin(theta) c(b) a_b to b xor x.
// Readings: a term with x != 0 is a branching operation (T_eps afterwards, the
// cap rule 2*nnz > cap skips it); a term with x == 0 is diagonal, a phase gate
// that never prunes and ignores the cap.
namespace {

struct PauliRecord {      // 64 bytes, little endian
  uint64_t x_lo, x_hi, z_lo, z_hi, ctrl_lo, ctrl_hi;
  double theta;
  uint64_t cap;
};
static_assert(sizeof(PauliRecord) == 64, "Pauli record layout");

// c(b): X = [[0,1],[1,0]], Y = [[0,-i],[i,0]], Z = [[1,0],[0,-1]], entry in
// row (bit xor x-bit), column (bit).
Amp pauli_coef(const PauliRecord& p, const Label& b, unsigned n_qubits) {
  const Label x{p.x_lo, p.x_hi}, z{p.z_lo, p.z_hi};
  Amp c{1.0, 0.0};
  for (unsigned q = 0; q < n_qubits; ++q) {
    const bool xq = bit_of(x, q), zq = bit_of(z, q), v = bit_of(b, q);
    Amp e;
    if (xq && zq)
      e = v ? Amp{0.0, -1.0} : Amp{0.0, 1.0};   // Y|0> = i|1>, Y|1> = -i|0>
    else if (xq)
      e = Amp{1.0, 0.0};                          // X
    else if (zq)
      e = v ? Amp{-1.0, 0.0} : Amp{1.0, 0.0};     // Z
    else
      continue;
    c = mul(c, e);
  }
  return c;
}

void accumulate(State& s, const Label& k, const Amp& a) {
  auto r = s.emplace(k, a);
  if (!r.second) r.first->second = add(r.first->second, a);
}

void apply_pauli_exp(Oracle& o, const PauliRecord& p) {
  const Label ctrl{p.ctrl_lo, p.ctrl_hi};
  const bool branching = p.x_lo != 0 || p.x_hi != 0;
  const Amp cos_t{std::cos(p.theta), 0.0};
  const Amp misin_t{0.0, -std::sin(p.theta)};     // -i sin(theta)
  State out;
  out.reserve(o.psi.size() * (branching ? 2 : 1));
  for (const auto& kv : o.psi) {
    const Label& b = kv.first;
    if (!controls_set(b, ctrl)) {
      accumulate(out, b, kv.second);
      continue;
    }
    accumulate(out, b, mul(cos_t, kv.second));
    const Label bx{b.lo ^ p.x_lo, b.hi ^ p.x_hi};
    accumulate(out, bx, mul(mul(misin_t, pauli_coef(p, b, o.n_qubits)), kv.second));
  }
  if (branching) prune(o, out);
  o.psi.swap(out);
}

bool pauli_valid(const Oracle& o, const PauliRecord& p) {
  Label lim{~0ull, ~0ull};
  if (o.n_qubits < 128)
    lim = o.n_qubits >= 64 ? Label{~0ull, o.n_qubits == 64 ? 0ull : ((1ull << (o.n_qubits - 64)) - 1)}
                           : Label{(1ull << o.n_qubits) - 1, 0ull};
  const uint64_t all_lo = p.x_lo | p.z_lo | p.ctrl_lo, all_hi = p.x_hi | p.z_hi | p.ctrl_hi;
  if ((all_lo & ~lim.lo) || (all_hi & ~lim.hi)) return false;
  if (((p.x_lo | p.z_lo) & p.ctrl_lo) || ((p.x_hi | p.z_hi) & p.ctrl_hi)) return false;
  return std::isfinite(p.theta);
}

}  // namespace

// Apply n Pauli-exponential terms in order.  trace (optional) as for orc_run
// (applied = 0 for a skipped branching term).  Returns 0 or -1 (invalid term
// at index *bad; the terms before it are applied).
int orc_run_pauli(void* h, const PauliRecord* terms, uint64_t n, Trace* trace, uint64_t* bad) {
  Oracle& o = *static_cast<Oracle*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const PauliRecord& p = terms[i];
    if (!pauli_valid(o, p)) {
      if (bad) *bad = i;
      return -1;
    }
    Trace tr{o.psi.size(), 1, -1, 0.0, 0.0};
    const bool branching = p.x_lo != 0 || p.x_hi != 0;
    if (branching && p.cap != 0 && 2 * o.psi.size() > p.cap) {
      tr.applied = 0;
      o.tot.u2_skipped++;
    } else {
      o.tot.updates += o.psi.size();
      if (branching)
        o.tot.u2_applied++;
      else
        o.tot.mono_gates++;
      apply_pauli_exp(o, p);
      note_peak(o);
    }
    if (trace) trace[i] = tr;
  }
  return 0;
}

// Export sorted ascending by (hi, lo).  Returns nnz; writes min(nnz, cap).
uint64_t orc_export(void* h, uint64_t* lo, uint64_t* hi, double* amp, uint64_t cap) {
  Oracle& o = *static_cast<Oracle*>(h);
  const auto v = sorted_entries(o.psi);
  for (uint64_t i = 0; i < v.size() && i < cap; ++i) {
    lo[i] = v[i].first.lo;
    hi[i] = v[i].first.hi;
    amp[2 * i] = v[i].second.re;
    amp[2 * i + 1] = v[i].second.im;
  }
  return v.size();
}

int orc_probabilities(void* h, unsigned q, double* p0, double* p1) {
  Oracle& o = *static_cast<Oracle*>(h);
  if (q >= o.n_qubits) return -1;
  probabilities(o, q, p0, p1);
  return 0;
}

void orc_totals(void* h, Totals* t) { *t = static_cast<Oracle*>(h)->tot; }

// Apply phase/permutation ops to independent (label, amplitude) samples, one
// at a time -- f and g composed per label exactly as in a queued run.  Any
// non-monomial op is an error (-1).  Used to check full-size runs on samples.
int orc_monomial_samples(const OpRecord* ops, uint64_t n_ops, uint64_t* lo, uint64_t* hi, double* amp,
                         uint64_t count) {
  std::vector<Monomial> run;
  run.reserve(n_ops);
  for (uint64_t i = 0; i < n_ops; ++i) {
    if (!is_monomial(ops[i].kind)) return -1;
    run.push_back(monomial_of(ops[i]));
  }
  for (uint64_t j = 0; j < count; ++j) {
    Label k{lo[j], hi[j]};
    Amp a{amp[2 * j], amp[2 * j + 1]};
    for (const Monomial& g : run) apply_monomial(g, k, a);
    lo[j] = k.lo;
    hi[j] = k.hi;
    amp[2 * j] = a.re;
    amp[2 * j + 1] = a.im;
  }
  return 0;
}

}  // extern "C"
