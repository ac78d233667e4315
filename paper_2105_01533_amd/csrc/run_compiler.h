// Host-side compilation of phase/permutation runs, shared by the single-state
// engine (sim_api.hip) and the batched server (serve.hip).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sparsesim.h"
#include "sim_internal.h"

namespace sparsesim {

// Per-entry kernel descriptor of a MONO op.
MonoDesc mono_desc(const sim_gate& g);

// The kernel descriptor of a validated SIM_OP_U2 gate (x = 0 -> the target bit).
U2Desc u2_desc(const sim_gate& g, double eps);

// Structural validity of an op for a state of n_qubits (qubits in range,
// target not a control, measurement arguments, finite coefficients).
bool gate_valid(uint32_t n_qubits, const sim_gate& g, std::string* why);

bool key_fits(uint32_t n_qubits, uint64_t lo, uint64_t hi);

// What the bit-sliced pass needs to know about one MONO op.
struct BsGateInfo {
  bool eligible, phase, turns;
  uint8_t words_read, words_write, g_omega;
  uint64_t g_turn;
};

// Bytecode of a list of MONO ops (in op order) and the per-run parameters.
struct RunCompiler {
  uint32_t n_qubits = 0;
  std::vector<MonoDesc> descs;      // one per MONO op
  std::vector<BsOp> ops;            // bit-sliced bytecode of all MONO ops
  std::vector<uint32_t> start;      // ops of MONO op k: [start[k], start[k+1])
  std::vector<BsGateInfo> info;
  std::vector<std::vector<BsOp>> part_ops;   // compile's per-thread output, kept between calls
  // Ops a pair attempt looks ahead over.  Wider finds more pairs (faster
  // passes) at more host time; the batched server, which groups on its
  // critical path, uses a narrower one.
  uint32_t pair_window = 128;

  // Fill ops/start/info from descs.
  void compile(uint32_t nq);
  // Whether MONO ops [begin, begin+len) run bit-sliced under the policy, and
  // the run parameters (bytes_per_entry left 0).
  bool run_params(size_t begin, size_t len, uint32_t mono_mode, uint32_t min_gates, BsRun* br) const;
  // Kernel ops of MONO ops [begin, begin+len), in groups of kBsGroup, appended
  // to out; the run constants of br (from run_params) take the phase the
  // rewrite of uncontrolled X gates moves into them.
  void group(size_t begin, size_t len, std::vector<BsGroup>& out, BsRun* br) const;
  // The ops with uncontrolled X gates carried to the end of the run, and the
  // eighth turns and turns that become run constants.
  void defer_x(const BsOp* in, uint32_t n, std::vector<BsOp>& out, uint32_t* d_omega, uint64_t* d_turn) const;
  // Groups of n bit-sliced ops, appended to out.
  void group_range(const BsOp* src, uint32_t n, std::vector<BsGroup>& out) const;
  // Register-plane program of MONO ops [begin, begin+len) (segments of one
  // shape), appended to out; br as for group().
  void schedule(size_t begin, size_t len, std::vector<RpRec>& out, BsRun* br) const;
  // Segments of n bit-sliced ops, appended to out.
  void schedule_range(const BsOp* src, uint32_t n, std::vector<RpRec>& out) const;
  // Records the program of n_ops bit-sliced ops on nq qubits may take at most
  // (the rewrite of uncontrolled X gates at most doubles the ops and adds nq;
  // a segment adds a header and up to three padding ops).
  static size_t rp_records_bound(size_t n_ops, uint32_t nq) { return 8 * (2 * n_ops + nq) + 16; }
};

}  // namespace sparsesim
