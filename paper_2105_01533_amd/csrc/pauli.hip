// Pauli exponentials exp(-i theta P), optionally controlled (Sec. 3 lists them
// among the intrinsic operations with at most two nonzeros per row), turned
// into the library's ops on the host.
//
// With P^2 = I the term is cos(theta) I - i sin(theta) P, and P|b> =
// c(b)|b ^ x> with c(b) = i^popcount(x & z) (-1)^popcount(b & z) (each Y
// contributes i (-1)^bit, each Z (-1)^bit, each X 1).  A term with x != 0 is
// one branching op: partner b ^ x, pivot the lowest bit of x, and for the pair
// (b0 with the pivot clear, b1 = b0 ^ x)
//   alpha'_b0 = cos alpha_b0 - i sin c(b1) alpha_b1
//   alpha'_b1 = cos alpha_b1 - i sin c(b0) alpha_b0,
// where c(b0) = i^ny s and c(b1) = i^ny (-1)^ny s with ny = popcount(x & z) and
// s = (-1)^popcount(b0 & z): the label-independent parts go into U, the sign s
// is applied per pair by the kernels.  A term with x == 0 is diagonal,
// e^{-i theta (-1)^popcount(b & z)}: a phase on the parity of the z qubits,
// which CNOTs gather onto one qubit inside a fused phase/permutation run.
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sparsesim.h"
#include "run_compiler.h"
#include "sim_internal.h"

namespace {

using sparsesim::key_fits;

uint32_t lowest_bit(uint64_t lo, uint64_t hi) {
  return lo ? (uint32_t)__builtin_ctzll(lo) : 64u + (uint32_t)__builtin_ctzll(hi);
}

sim_gate mono_gate(uint32_t target, uint64_t ctrl_lo, uint64_t ctrl_hi) {
  sim_gate g;
  std::memset(&g, 0, sizeof g);
  g.op = SIM_OP_MONO;
  g.target = target;
  g.ctrl.lo = ctrl_lo;
  g.ctrl.hi = ctrl_hi;
  g.forced = -1;
  g.m[0] = g.m[1] = sim_c64{1.0, 0.0};
  return g;
}

sim_gate cnot(uint32_t control, uint32_t target) {
  sim_gate g = mono_gate(target, control < 64 ? 1ull << control : 0ull, control >= 64 ? 1ull << (control - 64) : 0ull);
  g.flip = 1;
  return g;
}

bool term_valid(const sim_pauli& t, uint32_t n) {
  if (!key_fits(n, t.x.lo, t.x.hi) || !key_fits(n, t.z.lo, t.z.hi) || !key_fits(n, t.ctrl.lo, t.ctrl.hi)) return false;
  if (((t.x.lo | t.z.lo) & t.ctrl.lo) || ((t.x.hi | t.z.hi) & t.ctrl.hi)) return false;
  return std::isfinite(t.theta);
}

size_t ops_of(const sim_pauli& t) {
  if (t.x.lo || t.x.hi) return 1;
  const size_t k = (size_t)__builtin_popcountll(t.z.lo) + (size_t)__builtin_popcountll(t.z.hi);
  return k ? 2 * k - 1 : 1;
}

void emit(const sim_pauli& t, sim_gate* out) {
  const double c = std::cos(t.theta), s = std::sin(t.theta);
  if (t.x.lo || t.x.hi) {
    sim_gate g = mono_gate(lowest_bit(t.x.lo, t.x.hi), t.ctrl.lo, t.ctrl.hi);
    g.op = SIM_OP_U2;
    g.x = t.x;
    g.z = t.z;
    g.cap = t.cap;
    const int ny = __builtin_popcountll(t.x.lo & t.z.lo) + __builtin_popcountll(t.x.hi & t.z.hi);
    // u10 = -i sin(theta) i^ny, exact for every ny mod 4.
    sim_c64 u10;
    switch (ny & 3) {
      case 0: u10 = sim_c64{0.0, -s}; break;
      case 1: u10 = sim_c64{s, 0.0}; break;
      case 2: u10 = sim_c64{0.0, s}; break;
      default: u10 = sim_c64{-s, 0.0}; break;
    }
    const sim_c64 u01 = (ny & 1) ? sim_c64{-u10.re, -u10.im} : u10;
    g.m[0] = sim_c64{c, 0.0};
    g.m[1] = u01;
    g.m[2] = u10;
    g.m[3] = sim_c64{c, 0.0};
    out[0] = g;
    return;
  }
  if (!t.z.lo && !t.z.hi) {
    // exp(-i theta I) on the controlled subspace: the factor e^{-i theta}.
    if (!t.ctrl.lo && !t.ctrl.hi) {
      sim_gate g = mono_gate(0, 0, 0);
      g.m[0] = g.m[1] = sim_c64{c, -s};
      out[0] = g;
    } else {
      const uint32_t q = lowest_bit(t.ctrl.lo, t.ctrl.hi);
      sim_gate g = mono_gate(q, t.ctrl.lo & ~(q < 64 ? 1ull << q : 0ull),
                             t.ctrl.hi & ~(q >= 64 ? 1ull << (q - 64) : 0ull));
      g.m[1] = sim_c64{c, -s};
      out[0] = g;
    }
    return;
  }
  const uint32_t p = lowest_bit(t.z.lo, t.z.hi);
  std::vector<uint32_t> others;
  for (int w = 0; w < 2; ++w)
    for (uint64_t m = w ? t.z.hi : t.z.lo; m; m &= m - 1) {
      const uint32_t q = (uint32_t)__builtin_ctzll(m) + 64u * w;
      if (q != p) others.push_back(q);
    }
  size_t k = 0;
  for (uint32_t q : others) out[k++] = cnot(q, p);
  sim_gate g = mono_gate(p, t.ctrl.lo, t.ctrl.hi);
  g.m[0] = sim_c64{c, -s};   // even parity: eigenvalue +1
  g.m[1] = sim_c64{c, s};
  out[k++] = g;
  for (size_t i = others.size(); i-- > 0;) out[k++] = cnot(others[i], p);
}

}  // namespace

namespace sparsesim {

size_t pauli_op_count(const sim_pauli* terms, size_t n) {
  size_t total = 0;
  for (size_t i = 0; i < n; ++i) total += ops_of(terms[i]);
  return total;
}

}  // namespace sparsesim

extern "C" int sim_gates_from_pauli(const sim_pauli* terms, size_t n, uint32_t n_qubits, sim_gate* out, size_t cap,
                                    size_t* n_out) {
  using sparsesim::set_error;
  if (!n_out || (n && !terms)) return set_error(SIM_E_ARG, "null argument");
  if (n_qubits < 1 || n_qubits > 128) return set_error(SIM_E_ARG, "n_qubits must be in 1..128");
  size_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    if (!term_valid(terms[i], n_qubits)) return set_error(SIM_E_ARG, "term " + std::to_string(i) + ": invalid term");
    total += ops_of(terms[i]);
  }
  *n_out = total;
  if (total > cap || (total && !out)) return set_error(SIM_E_BUFFER, "output holds fewer ops than needed");
  size_t k = 0;
  for (size_t i = 0; i < n; ++i) {
    emit(terms[i], out + k);
    k += ops_of(terms[i]);
  }
  return SIM_OK;
}
