// Gate commuting (Sec. 3.3, Fig. 1) as a host rewrite of a standard-gate list:
// the ops are passed through per-qubit H, Rx, Ry queues that sit behind the
// phase/permutation queue, and the output is the sequence of ops the queues
// send on, in order.  Applying the output (sim_apply_ops) is then the paper's
// queued simulation; no device work happens here.
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sparsesim.h"
#include "sim_internal.h"

namespace {

bool op_bit(const sim_op& o, uint32_t q) { return ((q < 64 ? o.ctrl_lo >> q : o.ctrl_hi >> (q - 64)) & 1ull) != 0; }

// What is pending on one qubit after the phase/permutation queue, in the order
// it acts: H (if hadamard), then Rx(rx), then Ry(ry).
struct Lane {
  bool hadamard = false, has_rx = false, has_ry = false;
  double rx = 0.0, ry = 0.0;
  bool any() const { return hadamard || has_rx || has_ry; }
};

struct Rewriter {
  uint32_t nq;
  std::vector<Lane> lane;
  std::vector<sim_op> queue;       // pending phase/permutation ops, in order
  std::vector<sim_op>& out;

  Rewriter(uint32_t n, std::vector<sim_op>& o) : nq(n), lane(n), out(o) {}

  static sim_op single(uint32_t kind, uint32_t t, double theta) {
    sim_op r{};
    r.kind = kind;
    r.target = t;
    r.param = theta;
    r.forced = -1;
    return r;
  }

  // Send the phase/permutation queue, then what is pending on the marked
  // qubits (ascending).
  void drain(const std::vector<char>& mark) {
    out.insert(out.end(), queue.begin(), queue.end());
    queue.clear();
    for (uint32_t q = 0; q < nq; ++q) {
      if (!mark[q]) continue;
      Lane& l = lane[q];
      if (l.hadamard) out.push_back(single(SIM_K_H, q, 0.0));
      if (l.has_rx) out.push_back(single(SIM_K_RX, q, l.rx));
      if (l.has_ry) out.push_back(single(SIM_K_RY, q, l.ry));
      l = Lane{};
    }
  }
  void drain_one(uint32_t q) {
    std::vector<char> mark(nq, 0);
    mark[q] = 1;
    drain(mark);
  }
  // The op's qubits: its target, then its controls (ascending).
  template <class F>
  static void for_qubits(const sim_op& o, F&& f) {
    f(o.target);
    for (int w = 0; w < 2; ++w)
      for (uint64_t m = w ? o.ctrl_hi : o.ctrl_lo; m; m &= m - 1) f((uint32_t)__builtin_ctzll(m) + 64u * w);
  }
  std::vector<char> marks_of(const sim_op& o) const {
    std::vector<char> mark(nq, 0);
    for_qubits(o, [&](uint32_t q) { mark[q] = 1; });
    return mark;
  }
  static void add_angle(bool& has, double& angle, double theta) {
    const double sum = has ? angle + theta : theta;
    has = sum != 0.0;   // an exact 0 leaves no gate
    angle = has ? sum : 0.0;
  }

  void feed(const sim_op& o) {
    const uint32_t t = o.target;
    const bool bare = o.ctrl_lo == 0 && o.ctrl_hi == 0 && o.cap == 0;
    Lane& l = lane[t];
    if (o.kind <= SIM_K_PHASE) {
      // Phase/permutation op.  Through a pending H on its target an X or Z
      // (controls allowed) turns into a Z or X; anything else pending on one
      // of its qubits is sent on first.
      bool need = false;
      auto blocks = [&](uint32_t q) {
        const Lane& m = lane[q];
        const bool through_h = q == t && (o.kind == SIM_K_X || o.kind == SIM_K_Z) && !m.has_rx && !m.has_ry;
        return m.has_rx || m.has_ry || (m.hadamard && !through_h);
      };
      for_qubits(o, [&](uint32_t q) { need |= blocks(q); });
      if (need) {
        std::vector<char> mark(nq, 0);
        for_qubits(o, [&](uint32_t q) { mark[q] = blocks(q); });
        drain(mark);
      }
      sim_op g = o;
      if (lane[t].hadamard) g.kind = o.kind == SIM_K_X ? SIM_K_Z : SIM_K_X;
      queue.push_back(g);
      return;
    }
    if (o.kind == SIM_K_H && bare) {
      if (l.has_rx) {   // no simple relation through Rx
        drain_one(t);
        lane[t].hadamard = true;
        return;
      }
      if (l.has_ry) l.ry = -l.ry;   // H Ry(a) = Ry(-a) H
      l.hadamard = !l.hadamard;     // H H = I
      return;
    }
    if (o.kind == SIM_K_RX && bare) {
      if (l.has_ry) drain_one(t);   // Ry would have to act before the Rx
      add_angle(lane[t].has_rx, lane[t].rx, o.param);
      return;
    }
    if (o.kind == SIM_K_RY && bare) {
      add_angle(l.has_ry, l.ry, o.param);
      return;
    }
    // Controlled or capped branching op, or a measurement: its qubits'
    // pending gates (and the queue) go first, then the op itself.
    drain(marks_of(o));
    out.push_back(o);
  }

  void finish() { drain(std::vector<char>(nq, 1)); }
};

bool valid(const sim_op& o, uint32_t nq) {
  if (o.kind > SIM_K_MEASURE || o.target >= nq) return false;
  if (op_bit(o, o.target)) return false;
  if (nq < 128) {
    const uint64_t lo_ok = nq >= 64 ? ~0ull : ((1ull << nq) - 1);
    const uint64_t hi_ok = nq <= 64 ? 0ull : (nq == 128 ? ~0ull : ((1ull << (nq - 64)) - 1));
    if ((o.ctrl_lo & ~lo_ok) || (o.ctrl_hi & ~hi_ok)) return false;
  }
  return true;
}

}  // namespace

extern "C" int sim_commute_ops(const sim_op* in, size_t n, uint32_t n_qubits, sim_op* out, size_t cap,
                               size_t* n_out) {
  using sparsesim::set_error;
  if (!n_out || (n && !in)) return set_error(SIM_E_ARG, "null argument");
  if (n_qubits < 1 || n_qubits > 128) return set_error(SIM_E_ARG, "n_qubits must be in 1..128");
  for (size_t i = 0; i < n; ++i)
    if (!valid(in[i], n_qubits)) return set_error(SIM_E_ARG, "op " + std::to_string(i) + ": invalid op");
  std::vector<sim_op> res;
  res.reserve(n);
  Rewriter rw(n_qubits, res);
  for (size_t i = 0; i < n; ++i) rw.feed(in[i]);
  rw.finish();
  *n_out = res.size();
  if (res.size() > cap || (res.size() && !out)) return set_error(SIM_E_BUFFER, "output holds fewer ops than needed");
  std::copy(res.begin(), res.end(), out);
  return SIM_OK;
}
