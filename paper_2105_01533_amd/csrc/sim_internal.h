// Internal declarations shared by the HIP kernels and the host engine of
// libsparsesim (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sparsesim.h"

namespace sparsesim {

// Record an error for sim_last_error; returns code (sim_api.hip).
int set_error(int code, const std::string& msg);

// Ops that sim_gates_from_pauli writes for these terms.
size_t pauli_op_count(const sim_pauli* terms, size_t n);

constexpr uint64_t kEmptySlot = ~0ull;   // hash index: free slot
constexpr uint32_t kNoPartner = ~0u;     // partner look-up miss
constexpr int kMaxBlocks = 8192;         // blocks of the chunked (ordered) kernels
// Entries per block of the chunked kernels: the two-pass branching count and
// write, and the measurement reduce and write.  The host sizes their grids
// from its bound on the entry count with these; the kernels keep the same
// block ranges whatever that bound was.
constexpr uint64_t kTwoPassChunk = 2048, kMeasChunk = 8192;

// One state buffer (structure of arrays).  key_hi is null for states of at
// most 64 qubits, whose labels fit in key_lo.
struct Buf {
  uint64_t* key_lo;
  uint64_t* key_hi;
  double2* amp;
};

// Fused phase/permutation gate, read wave-uniformly through the scalar cache.
struct MonoDesc {
  uint64_t ctrl_lo, ctrl_hi;
  uint32_t target;
  uint32_t flags;              // kHasPhase | kFlip
  uint32_t pad0, pad1;
  double2 m0, m1;              // factor for target bit 0 / 1 (before the flip)
};
static_assert(sizeof(MonoDesc) == 64, "MonoDesc is 64 bytes");
constexpr uint32_t kHasPhase = 1u, kFlip = 2u;
// Run-level flags of a fused pass: some gate multiplies amplitudes / flips labels.
constexpr uint32_t kRunPhase = 1u, kRunFlip = 2u;

// Bit-sliced pass bytecode: one op per plane update.
//   kBsFlip:  plane[target] ^= AND(control planes)
//   kBsOmega: 3-bit counter += arg (eighths of a turn) where the condition holds
//   kBsTurn:  per-entry turn accumulator += arg (turn * 2^64) where it holds
// condition = AND(control planes) [& plane[target] when cmode == 1].
constexpr uint8_t kBsFlip = 0, kBsOmega = 1, kBsTurn = 2;
constexpr int kBsMaxCtrl = 3;
struct BsOp {
  uint8_t op, target, nctrl, cmode;
  uint8_t ctrl[4];
  uint64_t arg;
};
static_assert(sizeof(BsOp) == 16, "BsOp is 16 bytes");

// Kernel form of BsOps: groups of kBsGroup ops whose members touch no plane
// another member writes, so a group's plane reads can all be in flight at
// once.  In each op the condition is the AND of three plane slots (p0, p1, p2;
// unused slots name the all-ones plane); a flip xors it into plane t.
//
// Group-major, 64 bytes per group: the a words of the four ops, their b words,
// then their turn fractions.  Packed so that a plane's LDS byte offset
// (plane * 256) is a mask or a shift-and-mask of a word:
//   a: bits 0-1 op, 2-4 k (omega eighths), 5-7 group shape (first op only),
//      8-15 t, 16-23 p0, 24-31 p1
//   b: bits 8-15 p2
// The shape tells the kernel that all four ops are flips with the same number
// of controls (X, CX, CCX: only those planes are read, all named by a), that
// they are all turn ops (TURN; padding ops have tau = 0), that they are all
// eighth-turn ops conditioned on their target bit only (OMEGA; padding ops
// have k = 0), or that the group is general (three condition slots; flips and
// eighth-turn phase ops), PHASE when it holds a phase op.
constexpr int kBsGroup = 4;
constexpr uint32_t kShapeGeneric = 0, kShapeX = 1, kShapeCX = 2, kShapeCCX = 3, kShapeTurn = 4, kShapePhase = 5,
                   kShapeOmega = 6;
// In a[1] of an X, CX, CCX or OMEGA group: the next group has the same shape
// and no plane conflict with this one, so the kernel applies the eight ops as
// one (all reads, then all writes).  Never set on the last group of a batch of 64
// (position 63 mod 64 in its run).
constexpr uint32_t kPairBit = 1u << 5;
// In a[1] of such a group instead: the next three groups too (sixteen ops,
// one burst of reads).  Never set where the four would cross a batch of 64.
constexpr uint32_t kQuadBit = 1u << 7;
// In a[1] of a TURN group: no op of the group has controls, so each op's
// condition is its target plane alone (the kernel reads only that plane).
constexpr uint32_t kBareBit = 1u << 6;
// LDS planes of a tile beyond the label planes: all-ones and scratch.  (The
// TURN groups' table of subset sums is a static LDS array, placed before the
// planes.)
constexpr uint32_t kExtraPlanes = 2;
struct BsGroup {
  uint32_t a[kBsGroup], b[kBsGroup];
  uint64_t tau[kBsGroup];
};
static_assert(sizeof(BsGroup) == 64, "BsGroup is 64 bytes");
__host__ __device__ constexpr uint32_t bs_pack_a(uint32_t op, uint32_t k, uint32_t t, uint32_t p0, uint32_t p1) {
  return op | (k << 2) | (t << 8) | (p0 << 16) | (p1 << 24);
}
__host__ __device__ constexpr uint32_t bs_pack_b(uint32_t p2) { return p2 << 8; }
__host__ __device__ constexpr uint32_t bs_shape(uint32_t a0) { return (a0 >> 5) & 7u; }

// Register-plane program (the fused pass with planes held in VGPRs): a list
// of 16-byte quads.  A segment header quad (shape | count << 8, 0, 0, 0) is
// followed by count quads of ops, all of one shape:
//   F1, F2, F3  flips with 1, 2, 3 control planes, four per quad, one word
//               each: t | c0 << 8 | c1 << 16 | c2 << 24; plane t ^= AND of the
//               controls (an uncontrolled X names the all-ones plane);
//   OB + k      (k = 1..7) eighth-turn ops adding k where plane t holds, four
//               per quad, one word each: t;
//   OG          general eighth-turn ops, two per quad: (cond, k, cond, k),
//               cond = t | c0 << 8 | c1 << 16 | c2 << 24, condition = AND of
//               those four planes;
//   TB, TG      turn ops in groups of four, three quads per group: the four
//               cond words, then the four 64-bit turn fractions (lo, hi
//               words); TB: condition = plane t alone (cond = t), TG: AND of
//               the four planes of cond.  count = groups.
// A zero header (END) ends the program; the kernel reads the program through
// a buffer resource that returns zeros past its end.  Planes nq, nq + 1,
// nq + 2 are all-ones, scratch and zero; padding ops name them so that they
// change nothing.
constexpr uint32_t kRpEnd = 0, kRpF1 = 1, kRpF2 = 2, kRpF3 = 3, kRpOG = 5, kRpTB = 6, kRpTG = 7, kRpOB = 8;
struct RpRec {
  uint32_t w[4];
};
static_assert(sizeof(RpRec) == 16, "RpRec is 16 bytes");

// Run-level parameters of a bit-sliced pass.
struct BsRun {
  uint32_t n_planes;           // LDS planes per wave (= qubit count)
  uint32_t n_gates;            // gates in the run (update accounting)
  uint32_t words_read;         // 32-bit label words to transpose in (bit w = qubits 32w..32w+31)
  uint32_t words_write;        // label words to write back
  uint32_t has_phase;          // amplitudes change
  uint32_t has_turns;          // some kBsTurn op (per-entry 64-bit accumulators)
  uint32_t g_omega;            // entry-independent eighths of a turn
  uint32_t bytes_per_entry;    // algorithmic bytes per entry (accounting)
  uint64_t g_turn;             // entry-independent turn fraction * 2^64
};

// Branching operation (Eq. 2 with coefficients that depend on the label),
// passed by value.  A label's partner is label ^ x; of a pair, b0 is the label
// whose pivot bit (target, a bit of x) is 0 and b1 = b0 ^ x:
//   alpha'_b0 = u0 alpha_b0 + s u1 alpha_b1,  alpha'_b1 = s u2 alpha_b0 + u3 alpha_b1,
// s = (-1)^popcount(b0 & z).  A single-qubit gate has x = the target bit, z = 0.
struct U2Desc {
  uint64_t ctrl_lo, ctrl_hi;
  uint64_t x_lo, x_hi;         // partner mask
  uint64_t z_lo, z_hi;         // off-diagonal sign mask
  uint32_t target, pad;        // pivot bit
  double eps;
  double2 u[4];                // row-major
};

// Device control block.
struct Ctl {
  uint64_t nnz[2];             // entries in buffer 0 / 1
  uint64_t updates;            // sum over applied gates of nnz at input
  uint64_t peak;
  uint64_t pruned;
  uint64_t mono_bytes;         // algorithmic bytes of the fused phase/permutation passes
  uint64_t mono_updates;       // gate-entry updates of the fused passes
  // Algorithmic bytes (entries read and written) of the branching count and
  // write passes and of the measurement reduce and write passes.
  uint64_t pass_bytes[5];      // index 4: the one-block (LDS-index) branching kernel
  // Partner index work of branching gates: entries inserted, CAS attempts
  // (inserts + collisions), partner look-ups, slots the look-ups read.
  uint64_t ix[4];
  uint32_t error;              // bit 0: a measurement had no valid outcome; bit 1: a chained scan gave up
                               // waiting; bit 2: the one-block branching kernel met a state too large for it
  uint32_t ticket;             // tile counter of the single-pass branching kernel (wraps)
  double pruned_mass;          // sum of |a|^2 of the entries T_eps dropped
  // Counters of a two-pass branching gate, staged by its count pass and
  // committed by the scan only if the output fits the capacity (a gate
  // rejected for capacity changes no counter).
  uint64_t st_updates, st_pruned;
  double st_mass;
};

// Per-measurement record written by the decide kernel.
struct MeasRec {
  double p0, p1, scale;
  int32_t outcome, pad;
};

// Scratch of the chunked kernels, kMaxBlocks entries each.
struct BlockScratch {
  uint32_t* tot;               // per-block emitted counts, scanned in place to offsets
  uint32_t* tot2;              // measurement: the other offsets array (consecutive measurements alternate)
  uint32_t* cnt1;              // measurement: per-block count of labels with the qubit set
  double2* part;               // measurement: per-block (P0, P1)
};

// ---- batched execution (many states per launch) -----------------------------
// A tick applies one segment (a fused run, a branching gate or a measurement)
// to every active state.  Work is cut into units of kChunk entries of one
// state, so a state's results never depend on which other states share the
// launch.
constexpr uint32_t kChunk = 2048;          // entries per unit (= one bit-sliced tile)
constexpr uint32_t kFillUnit = 8192;       // index slots per fill unit
constexpr uint32_t kMaxPlanes = 128 + kExtraPlanes;   // label planes + all-ones, scratch
constexpr uint32_t kStOverflow = 1u, kStMeasure = 2u;
// Consecutive measurements of one state that one tick can run (one launch
// round each).
constexpr uint32_t kMaxChain = 8;

// Per-state control words, one slot each, read back after every tick.
struct SlotCtl {
  uint64_t nnz[2];
  MeasRec rec;
  int32_t outcome;
  uint32_t status;
  int32_t chain_out[kMaxChain];   // outcome of each measurement of a chain (-1: zero probability)
};
static_assert(sizeof(SlotCtl) == 88, "SlotCtl layout");

struct BItem {
  Buf in, out;                 // current and other buffer of the state
  SlotCtl* ctl;                // the state's control words
  uint32_t other;              // index of `out` in ctl->nnz
  uint32_t wide;
  uint64_t nnz;                // entries at input (exact)
  uint64_t cap;                // capacity of the state
  // fused run
  const BsGroup* gops;         // bit-sliced (LDS-plane) groups (gops != null) ...
  uint32_t ngroups, n_dops;
  const MonoDesc* dops;        // ... or per-entry descriptors
  BsRun run;
  uint32_t run_flags;
  uint32_t chain;              // measurement: its step in a chain of the tick (0: first; later steps
                               // take the entry count from ctl, at most nnz)
  // branching gate
  U2Desc u2;
  uint64_t* table;
  uint64_t mask;
  uint32_t* partner;
  uint32_t* tot;               // per-unit counts -> offsets; tot[units] = total
  // measurement
  uint32_t q;
  int32_t forced;
  double u;
  double2* part;
  uint32_t* cnt1;
};

// Tick header: item counts and the offsets (in uint32 words from the start
// of the unit table) of each family's first-unit arrays (length n + 1).
struct BTick {
  uint32_t n_mono, n_u2, n_meas;
  uint32_t n_u2s;              // small branching items (one block each, index in LDS), after the
                               // measurement items
  uint32_t mono_u0, fill_u0, build_u0, chunk_u0, meas_u0;
  uint32_t pad2[3];
};

// Kernel families of a tick: fused runs; branching gates on the global index;
// branching gates of small states (LDS index); measurements.
constexpr uint32_t kFamMono = 1, kFamU2 = 2, kFamU2s = 4, kFamMeas = 8, kFamAll = 15;
// The kernels of the families in `families`, in tick order.
void launch_batch_tick(hipStream_t st, const BTick* hdr, const BItem* items, const uint32_t* units, int grid,
                       uint32_t families);
// The measurement kernels alone (a later step of measurement chains).
void launch_batch_meas(hipStream_t st, const BTick* hdr, const BItem* items, const uint32_t* units, int grid);


// ---- launchers (sim_kernels.hip) -------------------------------------------
void launch_set_basis(hipStream_t st, Buf b, uint64_t* nnz, uint64_t lo, uint64_t hi);
void launch_mono(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const MonoDesc* g, uint32_t ng,
                 uint32_t run_flags, uint32_t bytes_per_entry, Ctl* ctl, int grid, int block);
void launch_mono_bs(hipStream_t st, Buf b, const uint64_t* nnz, const BsGroup* groups, uint32_t ngroups, const BsRun& run,
                    Ctl* ctl, int grid);
// Register-plane fused pass: one 2048-entry tile per block; grid covers the
// entry count's upper bound.
void launch_mono_rp(hipStream_t st, Buf b, const uint64_t* nnz, const RpRec* prog, uint32_t nrec, const BsRun& run,
                    Ctl* ctl, int grid);
// Set-up of the register-plane passes' cross-stream ordering on the current
// device (once per device; called by sim_create).
hipError_t mono_rp_init();
// n entries of a device state (key_lo, key_hi or null for <= 64 qubits, amp)
// into host key records and amplitudes, through the calling thread's pinned
// staging buffer; safe to call from several host threads at once.
hipError_t copy_state_to_host(const uint64_t* lo, const uint64_t* hi, const double2* amp, uint64_t n, sim_key* keys,
                              sim_c64* amps);
// The same into separate arrays (key_hi may be null: high words not wanted;
// zeros are written for a null hi).
hipError_t copy_state_to_host_soa(const uint64_t* lo, const uint64_t* hi, const double2* amp, uint64_t n,
                                  uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps);
void launch_fill(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n);
void launch_copy16(hipStream_t st, void* dst, const void* src, uint64_t n16);
// ctl: where the index counters go (Ctl::ix), or null to count nothing.
void launch_index_build(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, uint64_t* table, uint64_t mask,
                        const U2Desc& d, uint32_t* partner, Ctl* ctl, int grid, int block);
void launch_u2_probe(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const uint64_t* table, uint64_t mask,
                     const U2Desc& d, uint32_t* partner, Ctl* ctl, int grid, int block);
void launch_u2_count(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const U2Desc& d, const uint32_t* partner,
                     uint32_t* tot, Ctl* ctl, int grid, int block);
// cap: the count pass's staged counters are committed only if the total fits.
void launch_scan(hipStream_t st, uint32_t* tot, int nblocks, uint64_t* nnz_out, Ctl* ctl, uint32_t entry_bytes,
                 uint64_t cap);
void launch_u2_write(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const uint32_t* partner,
                     const uint32_t* off, const U2Desc& d, Ctl* ctl, int grid, int block);
// Entries per block of the single-pass branching kernel (512, 1024 or
// 2048); it serves states of at most kMaxBlocks tiles of the largest.
constexpr uint32_t kU2Tile = 2048;
// The tile for a state of at most ub entries: 512 up to 2^20 entries, 1024 up
// to kMaxBlocks such tiles, 2048 beyond.
inline uint32_t u2_tile_for(uint64_t ub) {
  return ub <= (1ull << 20) ? 512u : ub <= (uint64_t)kMaxBlocks * 1024u ? 1024u : kU2Tile;
}
// grid = tiles covering the entry count's bound.
void launch_u2_fused(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const uint32_t* partner,
                     const U2Desc& d, Ctl* ctl, uint64_t* status, uint32_t ticket_base, uint32_t epoch,
                     uint64_t* nnz_out, uint64_t* table, uint64_t clear_slots, int grid, uint32_t tile);
// Largest state the one-block branching kernel takes (its partner index and
// partner slots live in LDS).
constexpr uint32_t kLdsU2Max = 8192;
// One block: a branching gate on a state of at most kLdsU2Max entries, index
// and look-up in LDS; outputs, their order and the counters as the
// multi-kernel path's single pass (pruned_mass up to summation order).
void launch_u2_lds(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const U2Desc& d, Ctl* ctl,
                   uint64_t* nnz_out);
void launch_measure_reduce(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, uint32_t q, BlockScratch s,
                           int grid, int block);
void launch_measure_decide(hipStream_t st, const double2* part, const uint32_t* cnt1, uint32_t* off, int nblocks,
                           const uint64_t* nnz_in, uint64_t* nnz_out, double u, int32_t forced, MeasRec* rec,
                           int32_t* outcome, Ctl* ctl, uint32_t entry_bytes, const uint32_t* in_off);
void launch_measure_write(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, uint32_t q,
                          const MeasRec* rec, const uint32_t* off, const uint32_t* in_off, int32_t q_next,
                          double2* part_next, uint32_t* cnt1_next, int grid);

}  // namespace sparsesim
