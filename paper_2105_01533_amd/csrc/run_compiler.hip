// Host-side compilation of phase/permutation runs (see run_compiler.h).
#include "run_compiler.h"

#include "host_pool.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

namespace sparsesim {

MonoDesc mono_desc(const sim_gate& g) {
  MonoDesc d{};
  d.ctrl_lo = g.ctrl.lo;
  d.ctrl_hi = g.ctrl.hi;
  d.target = g.target;
  const bool unit = g.m[0].re == 1.0 && g.m[0].im == 0.0 && g.m[1].re == 1.0 && g.m[1].im == 0.0;
  d.flags = (unit ? 0u : kHasPhase) | (g.flip ? kFlip : 0u);
  d.m0 = make_double2(g.m[0].re, g.m[0].im);
  d.m1 = make_double2(g.m[1].re, g.m[1].im);
  return d;
}

bool key_fits(uint32_t n, uint64_t lo, uint64_t hi) {
  if (n >= 128) return true;
  if (n > 64) return (hi >> (n - 64)) == 0;
  return hi == 0 && (n == 64 || (lo >> n) == 0);
}

U2Desc u2_desc(const sim_gate& g, double eps) {
  U2Desc d{};
  d.ctrl_lo = g.ctrl.lo;
  d.ctrl_hi = g.ctrl.hi;
  const bool single = g.x.lo == 0 && g.x.hi == 0;
  d.x_lo = single ? (g.target < 64 ? 1ull << g.target : 0ull) : g.x.lo;
  d.x_hi = single ? (g.target >= 64 ? 1ull << (g.target - 64) : 0ull) : g.x.hi;
  d.z_lo = g.z.lo;
  d.z_hi = g.z.hi;
  d.target = g.target;
  d.eps = eps;
  for (int k = 0; k < 4; ++k) d.u[k] = make_double2(g.m[k].re, g.m[k].im);
  return d;
}

bool gate_valid(uint32_t n, const sim_gate& g, std::string* why) {
  if (g.op > SIM_OP_MEASURE) return *why = "unknown op class", false;
  if (g.target >= n || !key_fits(n, g.ctrl.lo, g.ctrl.hi)) return *why = "qubit out of range", false;
  const uint64_t tw = g.target < 64 ? g.ctrl.lo : g.ctrl.hi;
  if ((tw >> (g.target & 63)) & 1ull) return *why = "target is also a control", false;
  if (g.op == SIM_OP_U2) {
    if (!key_fits(n, g.x.lo, g.x.hi) || !key_fits(n, g.z.lo, g.z.hi)) return *why = "x or z out of range", false;
    if (((g.x.lo | g.z.lo) & g.ctrl.lo) || ((g.x.hi | g.z.hi) & g.ctrl.hi))
      return *why = "x or z meets the controls", false;
    const uint64_t xw = g.target < 64 ? g.x.lo : g.x.hi;
    if ((g.x.lo || g.x.hi) && !((xw >> (g.target & 63)) & 1ull)) return *why = "the target is not a bit of x", false;
  } else if (g.x.lo || g.x.hi || g.z.lo || g.z.hi) {
    return *why = "x and z are for branching ops only", false;
  }
  if (g.op == SIM_OP_MEASURE) {
    if (g.ctrl.lo || g.ctrl.hi) return *why = "measurement cannot be controlled", false;
    if (g.forced < -1 || g.forced > 1) return *why = "forced must be -1, 0 or 1", false;
    if (g.forced < 0 && !(g.u >= 0.0 && g.u < 1.0)) return *why = "measurement u must be in [0, 1)", false;
  } else {
    const int nm = g.op == SIM_OP_MONO ? 2 : 4;
    for (int k = 0; k < nm; ++k)
      if (!std::isfinite(g.m[k].re) || !std::isfinite(g.m[k].im)) return *why = "non-finite coefficient", false;
  }
  return true;
}

namespace {

// Exact eighth-turn factors omega^k = e^{i pi k / 4}; -1 if m is not one.
int omega_index(const double2& m) {
  const double h = M_SQRT1_2;
  const double re[8] = {1.0, h, 0.0, -h, -1.0, -h, 0.0, h};
  const double im[8] = {0.0, h, 1.0, h, 0.0, -h, -1.0, -h};
  for (int k = 0; k < 8; ++k)
    if (m.x == re[k] && m.y == im[k]) return k;
  return -1;
}

bool unit_modulus(const double2& m) { return std::fabs(m.x * m.x + m.y * m.y - 1.0) <= 1e-14; }

// Argument of m as a turn fraction in units of 2^-64 turn (wraps exactly).
uint64_t turn_of(const double2& m) {
  const long double tau = (long double)std::atan2(m.y, m.x) / (2.0L * (long double)M_PI);   // [-1/2, 1/2]
  long double v = tau * 18446744073709551616.0L;
  if (v >= 9223372036854775807.0L) v -= 18446744073709551616.0L;
  return (uint64_t)(int64_t)std::llroundl(v);
}

uint8_t word_bit(uint32_t q) { return (uint8_t)(1u << (q >> 5)); }

constexpr unsigned kHostThreads = HostPool::kMaxThreads;

}  // namespace

namespace {

// Bit-sliced ops of one MONO op, appended to out; inf describes them.
void compile_one(const MonoDesc& d, BsGateInfo& inf, std::vector<BsOp>& out) {
  inf.eligible = true;
  BsOp base{};
  base.target = (uint8_t)d.target;
  uint8_t rd = 0;
  for (int w = 0; w < 2; ++w) {
    uint64_t m = w ? d.ctrl_hi : d.ctrl_lo;
    while (m) {
      const uint32_t q = (uint32_t)__builtin_ctzll(m) + 64u * w;
      m &= m - 1;
      if (base.nctrl == kBsMaxCtrl) {
        inf.eligible = false;
        break;
      }
      base.ctrl[base.nctrl++] = (uint8_t)q;
      rd |= word_bit(q);
    }
  }
  if (!inf.eligible) return;
  auto emit = [&](uint8_t op, uint8_t cmode, uint64_t arg) {
    BsOp o = base;
    o.op = op;
    o.cmode = cmode;
    o.arg = arg;
    out.push_back(o);
    if (cmode) rd |= word_bit(d.target);
  };
  if (d.flags & kHasPhase) {
    const int k0 = omega_index(d.m0), k1 = omega_index(d.m1);
    if (k0 >= 0 && k1 >= 0) {
      if (k0) {
        if (base.nctrl == 0) inf.g_omega = (uint8_t)((inf.g_omega + k0) & 7);
        else emit(kBsOmega, 0, (uint64_t)k0);
      }
      const uint32_t dk = (uint32_t)(k1 - k0) & 7u;
      if (dk) emit(kBsOmega, 1, dk);
    } else if (unit_modulus(d.m0) && unit_modulus(d.m1)) {
      const uint64_t t0 = turn_of(d.m0), t1 = turn_of(d.m1);
      if (t0) {
        if (base.nctrl == 0) {
          inf.g_turn += t0;
        } else {
          emit(kBsTurn, 0, t0);
          inf.turns = true;
        }
      }
      if (t1 - t0) {
        emit(kBsTurn, 1, t1 - t0);
        inf.turns = true;
      }
    } else {
      inf.eligible = false;
      return;
    }
    inf.phase = true;
  }
  if (d.flags & kFlip) {
    emit(kBsFlip, 0, 0);
    inf.words_write = word_bit(d.target);
  }
  inf.words_read = rd;
}

}  // namespace

// Per op: a factor m0 on labels with the target bit 0 and m1 with it 1 equals
// m0 everywhere (under the controls) times m1/m0 where the target bit is 1.
// Large lists are compiled in parts on host threads.
void RunCompiler::compile(uint32_t nq) {
  n_qubits = nq;
  const size_t n_mono = descs.size();
  ops.clear();
  start.assign(n_mono + 1, 0);
  info.assign(n_mono, BsGateInfo{});
  part_ops.resize(kHostThreads);
  for (auto& v : part_ops) v.clear();
  std::vector<size_t> pb(kHostThreads, 0), pe(kHostThreads, 0);
  parallel_parts(n_mono, 16384, [&](size_t b, size_t e, size_t p) {
    // Appends go to a vector on this thread's stack (neighbouring vectors in
    // part_ops share cache lines); its storage is kept in part_ops between calls.
    std::vector<BsOp> out;
    out.swap(part_ops[p]);
    out.reserve(2 * (e - b));
    for (size_t k = b; k < e; ++k) {
      start[k] = (uint32_t)out.size();   // local to the part until the parts are joined
      compile_one(descs[k], info[k], out);
    }
    part_ops[p].swap(out);
    pb[p] = b;
    pe[p] = e;
  });
  size_t total = 0;
  for (auto& v : part_ops) total += v.size();
  ops.reserve(total);
  for (size_t p = 0; p < kHostThreads; ++p) {
    const uint32_t base = (uint32_t)ops.size();
    for (size_t k = pb[p]; k < pe[p]; ++k) start[k] += base;
    ops.insert(ops.end(), part_ops[p].begin(), part_ops[p].end());
  }
  start[n_mono] = (uint32_t)ops.size();
}

bool RunCompiler::run_params(size_t begin, size_t len, uint32_t mono_mode, uint32_t min_gates, BsRun* br) const {
  if (mono_mode == SIM_MONO_DIRECT) return false;
  if (mono_mode == SIM_MONO_AUTO && len < (min_gates ? min_gates : 16u)) return false;
  std::memset(br, 0, sizeof *br);
  uint32_t g_omega = 0;
  for (size_t k = begin; k < begin + len; ++k) {
    const BsGateInfo& g = info[k];
    if (!g.eligible) return false;
    br->words_read |= g.words_read | g.words_write;
    br->words_write |= g.words_write;
    br->has_phase |= g.phase ? 1u : 0u;
    br->has_turns |= g.turns ? 1u : 0u;
    g_omega += g.g_omega;
    br->g_turn += g.g_turn;
  }
  if (br->words_write & 3u) br->words_read |= 3u;
  if (br->words_write & 12u) br->words_read |= 12u;
  br->g_omega = g_omega & 7u;
  br->n_planes = n_qubits;
  br->n_gates = (uint32_t)len;
  return true;
}

// Pack the ops into groups of kBsGroup ops that touch no plane another member
// of the group writes (so the kernel may read all of a group's planes before
// any write), padding groups with no-op flips of the scratch plane.
//
// Ops are list-scheduled: an op may be taken ahead of earlier ops still
// waiting when it commutes with each of them, i.e. neither writes a plane the
// other reads or writes (phase accumulations commute exactly, so phase ops
// only conflict through the planes they read).  Among the ops of a window that
// may go next, groups whose four ops are flips with the same number of
// controls are preferred, because the kernel reads only those planes for them.
// Large runs are grouped in parts on host threads (ops never move between
// parts, so the parts' groups concatenate in order).
void RunCompiler::group(size_t begin, size_t len, std::vector<BsGroup>& out, BsRun* br) const {
  const uint32_t i0 = start[begin], i1 = start[begin + len];
  std::vector<BsOp> xo;
  uint32_t d_omega = 0;
  uint64_t d_turn = 0;
  defer_x(ops.data() + i0, i1 - i0, xo, &d_omega, &d_turn);
  if (br) {
    br->g_omega = (br->g_omega + d_omega) & 7u;
    br->g_turn += d_turn;
  }
  const uint32_t n = (uint32_t)xo.size();
  const size_t g0 = out.size();
  if (n < 2 * 2048) {
    group_range(xo.data(), n, out);
  } else {
    std::vector<std::vector<BsGroup>> parts(kHostThreads);
    parallel_parts(n, 2048, [&](size_t b, size_t e, size_t p) {
      std::vector<BsGroup> mine;   // on this thread's stack: the parts' vectors share cache lines
      group_range(xo.data() + b, (uint32_t)(e - b), mine);
      parts[p].swap(mine);
    });
    for (auto& v : parts) out.insert(out.end(), v.begin(), v.end());
  }
  // The kernel reads a run's groups 64 at a time and a pair's or quad's later
  // groups from the next lanes: where they would cross into the next batch,
  // the quad becomes pairs and single groups, the pair single groups (every
  // part is valid on its own).
  for (size_t p = g0; p < out.size(); ++p) {
    const size_t lane = (p - g0) % 64;
    if ((out[p].a[1] & kQuadBit) && lane > 60) {
      out[p].a[1] &= ~kQuadBit;
      for (size_t k = 0; k < 4; k += 2)
        if ((lane + k) % 64 != 63) out[p + k].a[1] |= kPairBit;
    }
    if ((out[p].a[1] & kPairBit) && lane == 63) out[p].a[1] &= ~kPairBit;
  }
}

// Uncontrolled X gates only relabel: instead of flipping a plane each time,
// a run carries them as a pending mask P (the stored plane q is the true
// bit q xor P_q) and applies what is left once, at the end of the run.  An op
// meeting a pending bit is rewritten, exactly:
//   * X on q: P_q ^= 1, no op;
//   * CNOT with a pending control: t ^= NOT c is t ^= c followed by an X on
//     t, so the CNOT stays and P_t toggles;
//   * a phase op conditioned on its target bit alone, the bit pending: adding
//     a where the bit is 0 equals adding a everywhere (a run constant) and -a
//     where it is 1;
//   * any other op with a pending control (or a controlled phase op with its
//     target pending): the pending X on those planes is applied first.
// A flip's own target may be pending: plane t ^= cond keeps t xor P_t right.
void RunCompiler::defer_x(const BsOp* in, uint32_t n, std::vector<BsOp>& out, uint32_t* d_omega,
                          uint64_t* d_turn) const {
  uint64_t P[2] = {0, 0};
  auto pending = [&](uint32_t q) { return ((P[q >> 6] >> (q & 63)) & 1ull) != 0; };
  auto toggle = [&](uint32_t q) { P[q >> 6] ^= 1ull << (q & 63); };
  auto apply_pending = [&](uint32_t q) {
    if (!pending(q)) return;
    BsOp x{};
    x.op = kBsFlip;
    x.target = (uint8_t)q;
    out.push_back(x);
    toggle(q);
  };
  out.reserve(n + n_qubits);
  for (uint32_t i = 0; i < n; ++i) {
    const BsOp& o = in[i];
    if (o.op == kBsFlip) {
      if (o.nctrl == 0) {
        toggle(o.target);
        continue;
      }
      if (o.nctrl == 1) {
        out.push_back(o);
        if (pending(o.ctrl[0])) toggle(o.target);
        continue;
      }
      for (int c = 0; c < o.nctrl; ++c) apply_pending(o.ctrl[c]);
      out.push_back(o);
      continue;
    }
    if (o.nctrl == 0 && o.cmode && pending(o.target)) {
      BsOp p = o;
      if (o.op == kBsOmega) {
        *d_omega += (uint32_t)o.arg;
        p.arg = (8u - (uint32_t)o.arg) & 7u;
      } else {
        *d_turn += o.arg;
        p.arg = 0ull - o.arg;
      }
      out.push_back(p);
      continue;
    }
    for (int c = 0; c < o.nctrl; ++c) apply_pending(o.ctrl[c]);
    if (o.cmode) apply_pending(o.target);
    out.push_back(o);
  }
  for (uint32_t q = 0; q < n_qubits; ++q) apply_pending(q);
}

void RunCompiler::group_range(const BsOp* src, uint32_t n, std::vector<BsGroup>& out) const {
  const uint32_t ones = n_qubits, scratch = n_qubits + 1;
  struct Mask {
    uint64_t lo = 0, hi = 0;
    void set(uint32_t q) { (q < 64 ? lo : hi) |= 1ull << (q & 63); }
    bool meets(const Mask& o) const { return ((lo & o.lo) | (hi & o.hi)) != 0; }
    void add(const Mask& o) {
      lo |= o.lo;
      hi |= o.hi;
    }
  };
  struct Item {
    Mask r, w;
    uint32_t shape;   // kShapeX/CX/CCX for flips with 0..2 controls, TURN, else kShapeGeneric
    uint32_t phase;
  };
  if (n == 0) return;
  std::vector<Item> items(n);
  // Pending ops as a doubly linked list in op order (index n = end).
  std::vector<uint32_t> nxt(n + 1), prv(n + 1);
  for (uint32_t i = 0; i < n; ++i) {
    const BsOp& o = src[i];
    Item& it = items[i];
    for (int c = 0; c < o.nctrl; ++c) it.r.set(o.ctrl[c]);
    if (o.cmode || o.op == kBsFlip) it.r.set(o.target);
    if (o.op == kBsFlip) it.w.set(o.target);
    it.phase = o.op != kBsFlip;
    it.shape = o.op == kBsTurn                           ? kShapeTurn
               : o.op == kBsFlip && o.nctrl <= 2          ? kShapeX + o.nctrl
               : o.op == kBsOmega && o.nctrl == 0 && o.cmode ? kShapeOmega
                                                          : kShapeGeneric;
    nxt[i] = i + 1;
    prv[i + 1] = i;
  }
  prv[0] = n;
  nxt[n] = 0;   // the list is 0 .. n-1; nxt[n] is the head
  auto unlink = [&](uint32_t j) {
    nxt[prv[j]] = nxt[j];
    prv[nxt[j]] = prv[j];
  };
  // Relative cost of one op slot in a group of each shape (LDS accesses plus
  // vector instructions in the kernel's group bodies).
  auto slot_cost = [](uint32_t shape) {
    return shape == kShapeX ? 4 : shape == kShapeCX ? 6 : shape == kShapeCCX ? 8 : shape == kShapeOmega ? 5 : 12;
  };
  constexpr uint32_t kWindow = 32;
  // Select up to kBsGroup ops from the first pending ops; `want` is a
  // shape all picks must have, or kShapeGeneric for any but turn ops (which
  // only go in TURN groups).
  // Turn ops are sparse but commute with every op that does not flip one of
  // their condition planes, so TURN groups look further ahead.
  // kAnyFlip12: flips with one or two controls, for CCX-shaped groups (a
  // CNOT's second control slot names the all-ones plane).
  constexpr uint32_t kAnyFlip12 = 0x100;
  auto select = [&](uint32_t want, uint32_t* sel, uint32_t cap) -> uint32_t {
    uint32_t k = 0, seen = 0;
    const uint32_t window = want == kShapeTurn ? 4 * kWindow : cap > (uint32_t)kBsGroup ? pair_window : kWindow;
    Mask gr, gw, br, bw;   // group reads / writes, reads / writes of ops passed over
    for (uint32_t j = nxt[n]; j != n && seen < window && k < cap; j = nxt[j], ++seen) {
      const Item& it = items[j];
      const bool shape_ok = want == kShapeGeneric ? it.shape != kShapeTurn
                            : want == kAnyFlip12  ? it.shape == kShapeCX || it.shape == kShapeCCX
                                                  : it.shape == want;
      const bool commutes = !it.w.meets(br) && !it.w.meets(bw) && !it.r.meets(bw);
      const bool fits = !it.w.meets(gr) && !it.w.meets(gw) && !it.r.meets(gw);
      if (shape_ok && commutes && fits) {
        sel[k++] = j;
        gr.add(it.r);
        gw.add(it.w);
      } else {
        br.add(it.r);
        bw.add(it.w);
      }
    }
    return k;
  };
  // Append a group of the picked ops (np <= kBsGroup), padded.
  auto emit = [&](const uint32_t* picked, uint32_t np, uint32_t shape) {
    uint32_t phase = 0;
    BsGroup grp;
    uint32_t u = 0;
    for (; u < np; ++u) {
      const uint32_t j = picked[u];
      unlink(j);
      phase |= items[j].phase;
      const BsOp& o = src[j];
      uint32_t slot[3] = {ones, ones, ones};
      for (int c = 0; c < o.nctrl; ++c) slot[c] = o.ctrl[c];
      const uint32_t t = (o.op == kBsFlip || o.cmode) ? o.target : ones;   // flip target, or a phase op's target-bit condition
      const uint32_t k = o.op == kBsOmega ? (uint32_t)(o.arg & 7u) : 0u;
      grp.a[u] = bs_pack_a(o.op, k, t, slot[0], slot[1]);
      grp.b[u] = bs_pack_b(slot[2]);
      grp.tau[u] = o.op == kBsTurn ? o.arg : 0;
    }
    for (; u < (uint32_t)kBsGroup; ++u) {
      if (shape == kShapeTurn) {
        grp.a[u] = bs_pack_a(kBsTurn, 0, ones, ones, ones);     // adds 0 turns
      } else if (shape == kShapeOmega) {
        grp.a[u] = bs_pack_a(kBsOmega, 0, ones, ones, ones);    // adds 0 eighths
      } else {
        grp.a[u] = bs_pack_a(kBsFlip, 0, scratch, ones, ones);  // scratch ^= ones, or scratch = ~scratch
      }
      grp.b[u] = bs_pack_b(ones);
      grp.tau[u] = 0;
    }
    grp.a[0] |= (shape == kShapeGeneric && phase ? kShapePhase : shape) << 5;
    if (shape == kShapeTurn) {
      bool bare = true;
      for (uint32_t v = 0; v < np; ++v) bare = bare && src[picked[v]].nctrl == 0;
      if (bare) grp.a[1] |= kBareBit;
    }
    out.push_back(grp);
  };
  const size_t base = out.size();
  uint32_t pick[4 * kBsGroup], best[kBsGroup];
  while (nxt[n] != n) {
    const uint32_t hs = items[nxt[n]].shape;
    const bool flip = hs == kShapeX || hs == kShapeCX || hs == kShapeCCX;
    // A flip or OMEGA group may join the next one or three groups: eight or
    // sixteen mutually independent ops of one shape, read together by the
    // kernel.
    // A Toffoli head gathers CNOTs too (their second control slot names the
    // all-ones plane), so that CCX-shaped groups pair and quad far more often.
    const uint32_t gshape = hs;
    uint32_t np = select(hs == kShapeCCX ? kAnyFlip12 : hs, pick, flip || hs == kShapeOmega ? 4 * kBsGroup : kBsGroup);
    if (np >= 2 * kBsGroup) {
      const uint32_t ng = np == 4 * kBsGroup ? 4 : 2;
      for (uint32_t k = 0; k < ng; ++k) {
        emit(pick + k * kBsGroup, kBsGroup, gshape);
        if (k == 0) out.back().a[1] |= ng == 4 ? kQuadBit : kPairBit;
      }
      // Picks beyond the emitted groups stay pending.
      continue;
    }
    np = std::min<uint32_t>(np, kBsGroup);
    uint32_t shape = hs;
    if (hs != kShapeGeneric && hs != kShapeTurn && np < (uint32_t)kBsGroup) {
      // A mixed general group may carry more ops than a padded uniform one
      // (an OMEGA head may also join a general group).
      const uint32_t nb = select(kShapeGeneric, best, kBsGroup);
      uint32_t s0 = items[best[0]].shape;
      for (uint32_t u = 1; u < nb; ++u)
        if (items[best[u]].shape != s0) s0 = kShapeGeneric;
      if ((double)slot_cost(s0) / nb < (double)slot_cost(hs) / np) {
        for (uint32_t u = 0; u < nb; ++u) pick[u] = best[u];
        np = nb;
        shape = s0;
      }
    }
    emit(pick, np, shape);
  }
  (void)base;
}

// Register-plane programs.  The kernel runs a segment's ops in order, so ops
// of one segment need not be independent; what a segment needs is length
// (one dispatch per segment).  Ops are list-scheduled: the first pending op
// opens a segment of its shape, and later pending ops of the same shape join
// it when they commute with every pending op they pass (neither writes a
// plane the other reads or writes; phase accumulations commute exactly).
// Eighth-turn ops conditioned on their target alone all commute, so a
// segment of them is split by k into sub-segments (one add sequence each).
void RunCompiler::schedule(size_t begin, size_t len, std::vector<RpRec>& out, BsRun* br) const {
  const uint32_t i0 = start[begin], i1 = start[begin + len];
  std::vector<BsOp> xo;
  uint32_t d_omega = 0;
  uint64_t d_turn = 0;
  defer_x(ops.data() + i0, i1 - i0, xo, &d_omega, &d_turn);
  if (br) {
    br->g_omega = (br->g_omega + d_omega) & 7u;
    br->g_turn += d_turn;
  }
  const uint32_t n = (uint32_t)xo.size();
  if (n < 2 * 2048) {
    schedule_range(xo.data(), n, out);
  } else {
    std::vector<std::vector<RpRec>> parts(kHostThreads);
    parallel_parts(n, 2048, [&](size_t b, size_t e, size_t p) {
      std::vector<RpRec> mine;
      schedule_range(xo.data() + b, (uint32_t)(e - b), mine);
      parts[p].swap(mine);
    });
    for (auto& v : parts) out.insert(out.end(), v.begin(), v.end());
  }
}

void RunCompiler::schedule_range(const BsOp* src, uint32_t n, std::vector<RpRec>& out) const {
  const uint32_t ones = n_qubits, scratch = n_qubits + 1, zero = n_qubits + 2;
  struct Mask {
    uint64_t lo = 0, hi = 0;
    void set(uint32_t q) { (q < 64 ? lo : hi) |= 1ull << (q & 63); }
    bool meets(const Mask& o) const { return ((lo & o.lo) | (hi & o.hi)) != 0; }
    void add(const Mask& o) {
      lo |= o.lo;
      hi |= o.hi;
    }
  };
  struct Item {
    Mask r, w;
    uint32_t shape;   // kRpF1..F3, kRpOB (any k), kRpOG, kRpTB, kRpTG
  };
  if (n == 0) return;
  std::vector<Item> items(n);
  std::vector<uint32_t> nxt(n + 1), prv(n + 1);
  for (uint32_t i = 0; i < n; ++i) {
    const BsOp& o = src[i];
    Item& it = items[i];
    for (int c = 0; c < o.nctrl; ++c) it.r.set(o.ctrl[c]);
    if (o.cmode || o.op == kBsFlip) it.r.set(o.target);
    if (o.op == kBsFlip) it.w.set(o.target);
    const bool bare = o.nctrl == 0 && o.cmode;
    it.shape = o.op == kBsFlip    ? (o.nctrl <= 1 ? kRpF1 : o.nctrl == 2 ? kRpF2 : kRpF3)
               : o.op == kBsOmega ? (bare ? kRpOB : kRpOG)
                                  : (bare ? kRpTB : kRpTG);
    nxt[i] = i + 1;
    prv[i + 1] = i;
  }
  prv[0] = n;
  nxt[n] = 0;
  auto unlink = [&](uint32_t j) {
    nxt[prv[j]] = nxt[j];
    prv[nxt[j]] = prv[j];
  };
  // A condition word: the target (or all-ones) plane and three control slots.
  auto cond_word = [&](const BsOp& o) {
    uint32_t c[3] = {ones, ones, ones};
    for (int q = 0; q < o.nctrl; ++q) c[q] = o.ctrl[q];
    const uint32_t t = o.cmode ? (uint32_t)o.target : ones;
    return t | c[0] << 8 | c[1] << 16 | c[2] << 24;
  };
  auto header = [&](uint32_t shape, uint32_t count) { out.push_back(RpRec{{shape | count << 8, 0, 0, 0}}); };
  // Quads of one-word ops, padded with `pad` words.
  auto word_quads = [&](uint32_t shape, const std::vector<uint32_t>& words, uint32_t pad) {
    const uint32_t nq4 = ((uint32_t)words.size() + 3) / 4;
    header(shape, nq4);
    for (uint32_t q = 0; q < nq4; ++q) {
      RpRec r;
      for (uint32_t u = 0; u < 4; ++u) r.w[u] = 4 * q + u < words.size() ? words[4 * q + u] : pad;
      out.push_back(r);
    }
  };
  constexpr uint32_t kWindow = 256;
  std::vector<uint32_t> sel, words;
  sel.reserve(kWindow);
  words.reserve(kWindow);
  while (nxt[n] != n) {
    const uint32_t shape = items[nxt[n]].shape;
    sel.clear();
    Mask br, bw;   // reads / writes of the pending ops passed over
    uint32_t seen = 0;
    for (uint32_t j = nxt[n]; j != n && seen < kWindow; j = nxt[j], ++seen) {
      const Item& it = items[j];
      if (it.shape == shape && !it.w.meets(br) && !it.w.meets(bw) && !it.r.meets(bw)) {
        sel.push_back(j);
      } else {
        br.add(it.r);
        bw.add(it.w);
      }
    }
    for (uint32_t j : sel) unlink(j);
    const uint32_t ns = (uint32_t)sel.size();
    if (shape == kRpTB || shape == kRpTG) {
      const uint32_t ng = (ns + 3) / 4;
      header(shape, ng);
      for (uint32_t g = 0; g < ng; ++g) {
        RpRec cw;
        uint64_t tau[4] = {0, 0, 0, 0};
        for (uint32_t u = 0; u < 4; ++u) {
          const uint32_t k = 4 * g + u;
          if (k < ns) {
            cw.w[u] = cond_word(src[sel[k]]);
            tau[u] = src[sel[k]].arg;
          } else {
            cw.w[u] = zero | zero << 8 | zero << 16 | zero << 24;   // adds 0 turns
          }
        }
        out.push_back(cw);
        out.push_back(RpRec{{(uint32_t)tau[0], (uint32_t)(tau[0] >> 32), (uint32_t)tau[1], (uint32_t)(tau[1] >> 32)}});
        out.push_back(RpRec{{(uint32_t)tau[2], (uint32_t)(tau[2] >> 32), (uint32_t)tau[3], (uint32_t)(tau[3] >> 32)}});
      }
      continue;
    }
    if (shape == kRpOG) {
      const uint32_t nq2 = (ns + 1) / 2;
      header(shape, nq2);
      for (uint32_t q = 0; q < nq2; ++q) {
        RpRec r;
        for (uint32_t h = 0; h < 2; ++h) {
          const uint32_t k = 2 * q + h;
          r.w[2 * h] = k < ns ? cond_word(src[sel[k]]) : (zero | zero << 8 | zero << 16 | zero << 24);
          r.w[2 * h + 1] = k < ns ? (uint32_t)src[sel[k]].arg & 7u : 0u;
        }
        out.push_back(r);
      }
      continue;
    }
    if (shape == kRpOB) {
      // All commute: one sub-segment per k (padding ops read the zero plane).
      for (uint32_t k = 1; k < 8; ++k) {
        words.clear();
        for (uint32_t j : sel)
          if (((uint32_t)src[j].arg & 7u) == k) words.push_back(src[j].target);
        if (!words.empty()) word_quads(kRpOB + k, words, zero);
      }
      continue;
    }
    words.clear();
    for (uint32_t j : sel) {
      const BsOp& o = src[j];
      uint32_t c[3] = {ones, ones, ones};
      for (int q = 0; q < o.nctrl; ++q) c[q] = o.ctrl[q];
      words.push_back((uint32_t)o.target | c[0] << 8 | c[1] << 16 | c[2] << 24);
    }
    // Padding: scratch ^= AND of zero planes (no change).
    word_quads(shape, words, scratch | zero << 8 | zero << 16 | zero << 24);
  }
}

}  // namespace sparsesim
