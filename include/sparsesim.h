/*
 * sparsesim.h -- C-ABI of the MI355X sparse state-vector simulator.
 *
 * Method: Jaques & Haner, "Leveraging state sparsity for more efficient
 * quantum simulations", arXiv 2105.01533.  A state sum_b alpha_b |b> is kept
 * as the list of its nonzero (label b, amplitude alpha_b) pairs (Sec. 3);
 * labels are 128-bit, qubit q is bit q of the label (Sec. 2.1), amplitudes
 * are FP64 complex.
 *
 * Device memory: the state lives in HBM as structure-of-arrays
 * (key_lo[], key_hi[], amp[] as interleaved re,im doubles), double-buffered
 * as in Sec. 3.1 (each operation that changes the entry count writes the
 * other buffer), plus a hash index used by branching gates.  All device work
 * is issued on the stream given at creation; nothing here creates streams.
 *
 * Conventions for every call:
 *   - return 0 (SIM_OK) on success, a negative SIM_E_* code on failure;
 *     sim_strerror() names the code, sim_last_error() gives detail;
 *   - a handle is not thread-safe; calls on one handle must not overlap;
 *   - host pointers are read or written only during the call;
 *   - on error the simulated state is unchanged unless stated otherwise.
 */
#ifndef SPARSESIM_H
#define SPARSESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_E_ARG (-1)      /* invalid argument (qubit out of range, bad op, duplicate key...) */
#define SIM_E_NOMEM (-2)    /* device or host allocation failed, or workspace too small */
#define SIM_E_CAPACITY (-3) /* the state would exceed the configured capacity */
#define SIM_E_BUFFER (-4)   /* caller buffer too small (required size reported) */
#define SIM_E_HIP (-5)      /* a HIP runtime call failed */
#define SIM_E_STATE (-6)    /* measurement of a zero-probability outcome, or empty state */

/* A basis-state label: qubit q is bit q of lo (q < 64) or bit q-64 of hi. */
typedef struct sim_key {
  uint64_t lo, hi;
} sim_key;

/* FP64 complex amplitude. */
typedef struct sim_c64 {
  double re, im;
} sim_c64;

/* Operation classes (Sec. 3.1: at most one nonzero per matrix row = MONO,
 * "monomial", i.e. a phase/permutation gate; two nonzeros = U2, "branching"). */
#define SIM_OP_MONO 0u
#define SIM_OP_U2 1u
#define SIM_OP_MEASURE 2u

/*
 * One operation (152 bytes).
 *
 * All ops: the op acts only on labels whose control bits (ctrl) are all set
 * (Sec. 2.1, controlled gates C^n U); ctrl must not contain the target bit
 * and every bit of ctrl and target must be < n_qubits.
 *
 * SIM_OP_MONO, a phase/permutation gate G(a|b>) = f(b) a |g(b)> (Sec. 3.2):
 *   on a label with controls set, the amplitude is multiplied by m[v] where v
 *   is the label's target bit before the gate, then the target bit is flipped
 *   if flip != 0.  When m[0] and m[1] are both exactly 1+0i no multiply is
 *   done.  Labels without the controls are unchanged.
 * SIM_OP_U2, a branching gate (Eq. 2; Sec. 3.1: the coefficients may depend
 *   on the label and the partner label is easy to compute): a label's
 *   partner is label ^ x, where x is the partner mask (x = 0 stands for the
 *   target bit alone); target is the pivot, a bit of x.  For each pair (b
 *   with the pivot bit 0, b' = b ^ x), with s = (-1)^popcount(b & z):
 *   alpha'_b = U00 alpha_b + s U01 alpha_b', alpha'_b' = s U10 alpha_b + U11
 *   alpha_b', absent partners counting as 0; m[0..3] is U row-major.  A
 *   single-qubit gate has x = 0 (or the target bit) and z = 0; a Pauli
 *   exponential has x and z from its Pauli string (sim_gates_from_pauli).
 *   Afterwards every entry with re*re + im*im < eps, or exactly zero, is
 *   dropped.  If cap != 0 the op is skipped when 2*nnz > cap (nnz before the
 *   op).  x and z must lie below n_qubits and not meet ctrl.
 * SIM_OP_MEASURE of qubit `target` (Sec. 2.1, Born rule): P0 and P1 are the
 *   summed |a|^2 over labels with the qubit 0 / 1; the outcome is `forced`
 *   if forced is 0 or 1, otherwise 0 iff u < P0/(P0+P1); labels with the
 *   other value are dropped and the rest scaled by 1/sqrt(P_outcome).
 * x and z are used by SIM_OP_U2 only and must be 0 for the other classes.
 */
typedef struct sim_gate {
  uint32_t op;
  uint32_t target;
  sim_key ctrl;
  uint32_t flip;
  int32_t forced;
  sim_c64 m[4];
  uint64_t cap;
  double u;
  uint64_t reserved;
  sim_key x;   /* SIM_OP_U2: partner mask */
  sim_key z;   /* SIM_OP_U2: off-diagonal sign mask */
} sim_gate;

/*
 * Standard-gate record (48 bytes), the format of generated circuits.
 * kind: SIM_K_*; param: rotation angle theta (RZ, RX, RY, PHASE) or the
 * uniform u in [0,1) for MEASURE; cap and forced as in sim_gate.
 * Gate matrices are those of Sec. 2.1: H = sqrt(.5)[[1,1],[1,-1]],
 * S = diag(1,i), Pauli X, Y, Z, R_P(theta) = exp(-i theta P / 2); T =
 * diag(1, e^{i pi/4}), the adjoints, and PHASE(theta) = diag(1, e^{i theta}).
 */
#define SIM_K_X 0u
#define SIM_K_Y 1u
#define SIM_K_Z 2u
#define SIM_K_S 3u
#define SIM_K_SDG 4u
#define SIM_K_T 5u
#define SIM_K_TDG 6u
#define SIM_K_RZ 7u
#define SIM_K_PHASE 8u
#define SIM_K_H 9u
#define SIM_K_RX 10u
#define SIM_K_RY 11u
#define SIM_K_MEASURE 12u

typedef struct sim_op {
  uint32_t kind;
  uint32_t target;
  uint64_t ctrl_lo, ctrl_hi;
  double param;
  uint64_t cap;
  int32_t forced;
  uint32_t pad;
} sim_op;

/*
 * Pauli-exponential term (64 bytes): exp(-i theta P), one of the intrinsic
 * operations of Sec. 3 (at most two nonzeros per row), optionally controlled.
 * P acts as X on the qubits in x only, as Y on those in both x and z, as Z on
 * those in z only, and as the identity elsewhere; Sec. 2.1's Pauli rotation
 * R_P(phi) is theta = phi / 2.  Since P^2 = I the term is cos(theta) I -
 * i sin(theta) P, and P|b> = c(b)|b ^ x> with c(b) = i^popcount(x & z)
 * (-1)^popcount(b & z).  A term with x != 0 is a branching operation (pruned
 * afterwards, skipped when cap != 0 and 2*nnz > cap); a term with x == 0 is
 * a phase gate (no pruning, cap ignored).  x, z and ctrl must lie below
 * n_qubits, and ctrl must not meet x or z.
 */
typedef struct sim_pauli {
  sim_key x;
  sim_key z;
  sim_key ctrl;
  double theta;
  uint64_t cap;
} sim_pauli;

/* Creation parameters. Zero fields take the stated defaults. */
typedef struct sim_config {
  uint32_t n_qubits;    /* 1..128 */
  uint32_t fuse_max;    /* max phase/permutation gates per fused pass (default 65536) */
  uint64_t capacity;    /* max entries the state may hold, < 2^31 (required) */
  double eps;           /* prune threshold on |a|^2 after branching gates (0 = drop exact zeros only) */
  double load_factor;   /* hash index target load, (0, 0.9] (default 0.5) */
  uint32_t block;       /* threads per block of the per-entry fused pass: 64, 128 or 256 (default 256) */
  uint32_t flags;       /* SIM_FLAG_* bits; others must be 0 */
  uint32_t mono_mode;   /* fused-pass kernel: SIM_MONO_AUTO, SIM_MONO_DIRECT or SIM_MONO_BITSLICE */
  uint32_t bs_min_gates; /* SIM_MONO_AUTO: bit-sliced pass for runs of at least this many gates (default 16) */
} sim_config;

/* Branching gates whose outputs are known to fit the capacity run as one
 * pass (evaluation, a chained scan over 2048-entry tiles, and the ordered
 * write in one kernel) on states of up to 2^24 entries; this flag makes them
 * run as separate count, scan and write passes instead.  The results are
 * identical. */
#define SIM_FLAG_U2_TWO_PASS 1u

/* The bit-sliced fused pass keeps a tile's label bit-planes in VGPRs and
 * addresses them by index (the default); this flag selects the form that
 * keeps them in LDS instead.  The results are identical. */
#define SIM_FLAG_BS_LDS 2u

/* Branching gates on small states (at most 8192 entries) run as one block
 * whose partner index is in LDS; this flag sends them through the global
 * index (index build, probe, single pass) like larger states.  Both give the
 * same outputs in the same order. */
#define SIM_FLAG_U2_GLOBAL_INDEX 4u

/* Count the global index's work (sim_stats index_*): one atomic add per
 * block of the index-build and look-up kernels, so off by default.  The
 * one-block LDS-index kernel always counts (four adds per gate). */
#define SIM_FLAG_COUNT_INDEX 8u

/* The library tracks which qubits are the same in every entry (all, after
 * sim_set_basis; those the imported labels agree on after sim_import_state;
 * a flip keeps its target so only if its controls are; a branching gate takes
 * its partner-mask qubits out; a measurement puts its qubit back).  A
 * branching gate whose partner mask meets that set has no partners, so it
 * runs without building or probing an index.  This flag turns that off (the
 * results are the same).  The state must not be changed through the pointers
 * of sim_device_state. */
#define SIM_FLAG_NO_UNIFORM 16u

/* Fused phase/permutation pass variants.  DIRECT evaluates every gate on every
 * entry with sequential complex products (results bit-identical to a plain
 * sequential evaluation).  BITSLICE transposes 2048-entry tiles into bit-planes
 * (one 32-bit word per qubit per lane), applies permutations as plane
 * operations and accumulates phases exactly as turn fractions, multiplying
 * each amplitude once per run (results differ from sequential products by
 * rounding only).  It applies to runs whose gates have at most 3 controls and
 * unit-modulus factors; other runs use DIRECT. */
#define SIM_MONO_AUTO 0u
#define SIM_MONO_DIRECT 1u
#define SIM_MONO_BITSLICE 2u

/* Counters of one sim_apply_gates call (filled when stats != NULL). */
typedef struct sim_stats {
  uint64_t gates_applied;  /* ops consumed, including skipped branching gates */
  uint64_t updates;        /* sum over applied gates of nnz at the gate's input */
  uint64_t mono_passes;    /* fused phase/permutation kernel launches */
  uint64_t u2_applied, u2_skipped, measures;
  uint64_t host_syncs;     /* host waits for a device-computed nnz */
  uint64_t peak_nnz;       /* largest entry count reached */
  uint64_t pruned;         /* entries dropped by the eps rule */
  uint64_t bitslice_passes; /* fused passes that ran the bit-sliced kernel */
  double pruned_mass;      /* sum of |a|^2 of the dropped entries (summed in no fixed
                              order: equal to the oracle's to rounding); the batched
                              server counts neither pruned nor pruned_mass (0) */
  /* Partner-index work of the branching gates (Sec. 3.1): entries inserted,
   * insert CAS attempts (inserts + collisions), partner look-ups and the index
   * slots they read (probes / look-up is the mean probe length).  Always
   * counted for the one-block LDS index; for the global index only with
   * SIM_FLAG_COUNT_INDEX.  CAS attempts and probes depend on the order in
   * which threads insert, so they vary from run to run; the batched server
   * does not count them (0). */
  uint64_t index_inserts, index_cas, index_lookups, index_probes;
  uint64_t u2_split;        /* of u2_applied: gates known to have no partners, run without the global
                               index (see SIM_FLAG_NO_UNIFORM) */
} sim_stats;

typedef struct sim_t sim_t;

/* Device bytes a state with this configuration uses (both entry buffers,
 * the hash index and per-entry scratch); the size of a caller workspace. */
size_t sim_workspace_bytes(const sim_config* cfg);

/* Create a simulator in state |0...0>.  stream: a hipStream_t (NULL = the
 * null stream).  workspace: device memory of at least sim_workspace_bytes(cfg)
 * bytes, borrowed (it must outlive the handle), or NULL to let the library
 * allocate it.  Errors: SIM_E_ARG (config), SIM_E_NOMEM, SIM_E_HIP. */
int sim_create(const sim_config* cfg, void* stream, void* workspace, size_t ws_bytes, sim_t** out);

/* Free what the library allocated; a borrowed workspace is left alone. */
int sim_destroy(sim_t* s);

/* Reset to the single basis state k with amplitude 1. */
int sim_set_basis(sim_t* s, sim_key k);

/* Replace the state by n host (key, amplitude) pairs, copied in.  Duplicate
 * keys or bits above n_qubits -> SIM_E_ARG; n > capacity -> SIM_E_CAPACITY. */
int sim_import_state(sim_t* s, const sim_key* keys, const sim_c64* amps, uint64_t n);

/* Convert n standard-gate records into sim_gate ops (host only). */
int sim_gates_from_ops(const sim_op* ops, size_t n, sim_gate* out);

/*
 * Apply n ops in order.  Consecutive MONO ops (and skipped U2 ops between
 * them, which leave nnz unchanged) are fused into passes of at most fuse_max
 * gates, each label taking all of them in turn (Sec. 3.2).  The host reads a
 * device-computed nnz only when a cap decision or the capacity check needs it.
 * outcomes (optional): one int32 per MEASURE op, in order.  stats optional.
 * Returns when all work is done.  SIM_E_CAPACITY: the state is the state
 * before the failing op and stats->gates_applied counts the ops before it.
 * SIM_E_ARG: an invalid op; nothing was applied.
 */
int sim_apply_gates(sim_t* s, const sim_gate* gates, size_t n, int32_t* outcomes, sim_stats* stats);

/*
 * sim_apply_gates for callers that cannot allocate memory (code that must not
 * call hipMalloc: graph-building or tight serving loops, harnesses that
 * forbid it).  Same arguments, semantics, results and errors as
 * sim_apply_gates (results are bitwise those of sim_apply_gates on the same
 * handle state), but the call allocates no device or pinned host memory and
 * creates no events or threads: the device buffers a call needs beyond the
 * state (phase/permutation descriptors, register-plane programs, measurement
 * records and outcomes) live in a 32 MiB static device array of the library,
 * one per GPU, held until the process ends; uploads go from the handle's host
 * buffers (pageable), whose capacity is kept between calls.  The handle must
 * already exist (sim_create allocates, or borrows a caller workspace) and
 * profiling events are not recorded during the call.  Limits: at most 65536
 * ops per call (more -> SIM_E_ARG, nothing applied; split the list), a
 * handle created with SIM_FLAG_BS_LDS -> SIM_E_ARG, and a single fused run
 * whose program exceeds the array -> SIM_E_NOMEM (the state is then that
 * before the run).  Calls on one GPU share its array: the library runs them
 * one at a time within a process (each returns only after its stream has
 * drained), so overlapping calls from threads of one process serialize.
 * Synchronizes, like sim_apply_gates.
 */
int sim_apply_gates_static(sim_t* s, const sim_gate* gates, size_t n, int32_t* outcomes, sim_stats* stats);

/*
 * Gate commuting (Sec. 3.3, Fig. 1), host only.  Passes n standard-gate
 * records through per-qubit queues of H, Rx and Ry gates that act after the
 * phase/permutation queue, and writes the ops the queues send on, in order,
 * to out (at most n of them; *n_out receives the count).  Relations used:
 * H Ry(a) = Ry(-a) H and H H = I for an incoming H; Rx and Ry angles add up
 * (an exact 0 sum leaves no gate); an incoming X or Z, possibly controlled,
 * whose target has an H pending becomes Z or X.  Where no relation applies,
 * the phase/permutation queue and then the H, Rx, Ry pending on the op's
 * qubits are sent first (qubits in ascending order); controlled or capped
 * branching ops and measurements are sent after that as they are; at the end
 * everything pending is sent.  Applying the output (sim_apply_ops) simulates
 * the circuit with the paper's queues; a capped op is then skipped or not
 * where it is applied.  SIM_E_ARG for an invalid op (nothing written);
 * SIM_E_BUFFER if cap is too small (*n_out set).
 */
int sim_commute_ops(const sim_op* in, size_t n, uint32_t n_qubits, sim_op* out, size_t cap, size_t* n_out);

/*
 * Convert n Pauli terms into sim_gate ops (host only), written to out (at
 * most cap of them; *n_out receives the count).  A term with x != 0 becomes
 * one SIM_OP_U2 op whose pivot is the lowest bit of x, with U = [[cos theta,
 * u01], [u10, cos theta]], u10 = -i sin(theta) i^popcount(x & z) and u01 =
 * u10 (-1)^popcount(x & z), and the term's x, z, ctrl and cap.  A term with
 * x == 0 and k > 0 qubits in z becomes 2k - 1 phase/permutation ops: CNOTs
 * from the other z qubits onto the lowest one, the controlled factor
 * diag(e^{-i theta}, e^{i theta}) there, and the CNOTs again; with z == 0 it
 * is the controlled global factor e^{-i theta} (one op).  At most 255 ops per
 * term.  SIM_E_ARG for an invalid term (nothing written); SIM_E_BUFFER if cap
 * is too small (*n_out set).
 */
int sim_gates_from_pauli(const sim_pauli* terms, size_t n, uint32_t n_qubits, sim_gate* out, size_t cap,
                         size_t* n_out);

/* sim_gates_from_pauli followed by sim_apply_gates (no measurements). */
int sim_apply_pauli(sim_t* s, const sim_pauli* terms, size_t n, sim_stats* stats);

/* sim_gates_from_ops followed by sim_apply_gates. */
int sim_apply_ops(sim_t* s, const sim_op* ops, size_t n, int32_t* outcomes, sim_stats* stats);

/* Measure one qubit (u, forced as for SIM_OP_MEASURE); writes the outcome
 * and P1/(P0+P1) before collapse.  Synchronizes. */
int sim_measure(sim_t* s, uint32_t qubit, double u, int32_t forced, int32_t* outcome, double* p1);

/* Current number of stored entries.  Synchronizes. */
int sim_nnz(sim_t* s, uint64_t* nnz);

/* Wait for all work issued on the handle's stream. */
int sim_sync(sim_t* s);

/* Copy the state to caller-owned host arrays of `cap` entries, in storage
 * order (unsorted).  *nnz receives the entry count; if cap < nnz nothing is
 * copied and SIM_E_BUFFER is returned.  Synchronizes. */
int sim_export_state(sim_t* s, sim_key* keys, sim_c64* amps, uint64_t cap, uint64_t* nnz);

/* The same into separate arrays: key_lo[i] and key_hi[i] are the low and
 * high 64 bits of entry i's label (key_hi may be NULL when the high words are
 * not wanted; zeros for <= 64 qubits), amps[i] its amplitude.  Arrays of cap
 * entries, caller-owned; sizes and errors as sim_export_state. */
int sim_export_state_soa(sim_t* s, uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps, uint64_t cap, uint64_t* nnz);

/* Device addresses of the current state buffers (key_lo, key_hi, amp) and
 * the device nnz word, for zero-copy inspection (read only); valid until the
 * next call. */
int sim_device_state(sim_t* s, uint64_t** key_lo, uint64_t** key_hi, double** amp, uint64_t** d_nnz);

/* Per-kernel-class counters, cumulative since creation or the last reset.
 * The kernel classes are mono_pass, index_fill, index_build, u2_probe,
 * u2_count, block_scan, u2_write (the single-pass branching kernel counts
 * here; u2_count and block_scan run only in the two-pass form),
 * measure_reduce, measure_decide and measure_write (a chain of consecutive
 * measurements runs one reduce), and u2_lds (the one-block branching kernel
 * of states of at most 8192 entries, index in LDS).
 * With profiling on for a class (sim_set_profiling), every launch of it is
 * bracketed by HIP events on the handle's stream and total_ms sums their
 * elapsed times; otherwise total_ms is 0.  alg_bytes is the algorithmic HBM
 * traffic of a class, the bytes its pass must move at least: for the fused
 * phase/permutation pass the label read, label write if any gate flips and
 * amplitude read+write if any gate has a phase; for u2_count every input
 * entry read; for u2_write every input entry read and every output entry
 * written, and the same for u2_lds; for measure_reduce the label word holding the measured qubit and the
 * amplitude of every entry; for measure_write that label word of every entry, the
 * rest of each kept entry and the kept entries written; 0 for the others
 * (index, scan and decide work is overhead);
 * updates counts gate-entry updates done by the class.  Three host classes
 * follow the kernel classes, always measured on the host's wall clock:
 * host_prepare (validation and op compilation at the start of a call),
 * host_group (grouping of bit-sliced runs) and host_sync (time blocked in
 * stream synchronisations); their launches count calls. */
typedef struct sim_kernel_stat {
  char name[32];
  uint64_t launches;
  double total_ms;
  double alg_bytes;
  double updates;
} sim_kernel_stat;

/* Change the launch tuning of a live handle: fuse_max, block, mono_mode and
 * bs_min_gates are taken from t (zero = default); load_factor is taken if it
 * is at least the creation value (the index was sized for that one); other
 * fields of t are ignored; flags is taken as well, except SIM_FLAG_BS_LDS,
 * which only sim_create sets (SIM_E_ARG here).  Results change only by
 * rounding (mono_mode) or not at all.  SIM_E_ARG on invalid values. */
int sim_set_tuning(sim_t* s, const sim_config* t);

/* Bandwidth reference: copy `bytes` (a multiple of 16) from device src to
 * device dst with a plain streaming kernel on `stream` (NULL = null stream);
 * asynchronous.  Used to calibrate hardware byte counters against a kernel
 * that moves a known number of bytes.  SIM_E_ARG for a bad size. */
int sim_device_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Profiling mode: SIM_PROFILE_OFF, SIM_PROFILE_ALL (every kernel launch is
 * bracketed by events) or SIM_PROFILE_MONO (only the fused phase/permutation
 * passes, for timing them with fewer events in flight).  Synchronises the
 * handle's stream.  SIM_E_ARG for another value. */
#define SIM_PROFILE_OFF 0
#define SIM_PROFILE_ALL 1
#define SIM_PROFILE_MONO 2
int sim_set_profiling(sim_t* s, int on);
/* Writes up to cap records; *n receives the number of classes. */
int sim_kernel_stats(sim_t* s, sim_kernel_stat* out, int cap, int* n);
int sim_kernel_stats_reset(sim_t* s);

/* ==== Continuous-batching server =========================================
 *
 * Many independent simulations share one device.  A request is a circuit
 * (sim_gate ops, as for sim_apply_gates) plus a sim_config (n_qubits,
 * capacity, eps, load_factor, fuse_max, mono_mode, bs_min_gates) and an
 * initial basis label.  Requests wait in FIFO order and are admitted while
 * their device footprint (srv_footprint) fits the pool and a slot is free; a
 * request larger than the whole pool is rejected at submission.  Each
 * srv_tick applies one segment (a fused phase/permutation run, one branching
 * gate or one measurement, cut exactly as sim_apply_gates cuts the circuit)
 * to every running request in one batched launch -- captured once as a
 * hipGraph and replayed every tick -- reads back every request's entry count
 * and measurement outcome, retires finished requests to host memory and
 * frees their device memory.  States stay device-resident between ticks.
 * A request's result does not depend on the other requests in the batch, and
 * equals a standalone sim_apply_gates run up to floating-point rounding of
 * the measurement sums and of the fused-pass kernel choice.
 * A server is not thread-safe; calls must not overlap.
 */
#define SRV_QUEUED 0
#define SRV_RUNNING 1
#define SRV_DONE 2
#define SRV_FAILED 3

#define SRV_FLAG_NO_GRAPH 1u /* launch the tick kernels directly instead of replaying the graph */
/* Branching gates of states of at most 8192 entries run one block per state
 * with the partner index in LDS; this flag sends them through the global
 * index kernels like larger states (same outputs, same order). */
#define SRV_FLAG_U2_GLOBAL_INDEX 2u
/* Bit-sliced fused runs of states of at least 65,536 entries run on the
 * register-plane kernel, one launch per run on the server's stream ahead of
 * the tick's graph; this flag keeps them on the graph's LDS-plane tile (the
 * same results, bit for bit). */
#define SRV_FLAG_NO_RP 4u
/* A branching gate or measurement that directly follows a request's fused
 * run joins the run's tick (the fused kernels run first, in place, and keep
 * the entry count): one host round trip for the pair instead of two; and up
 * to 8 consecutive measurements of a request run in one tick, one launch
 * round each, a later one taking its entry count from the device.  This flag
 * gives every request one segment per tick (the same results). */
#define SRV_FLAG_ONE_SEGMENT 8u

typedef struct srv_config {
  uint64_t budget_bytes; /* device bytes for request states (the pool) */
  uint64_t arena_bytes;  /* per-tick upload area for fused-run ops (0 = 64 MiB, else at least 1 MiB).
                            A fused run is never cut by the arena: runs are at most as long as fit
                            an empty arena, and a run that does not fit what a tick has left waits
                            whole for the next tick (first in line), so results do not depend on
                            the mix */
  uint32_t max_slots;    /* requests running at once, 1..4096 */
  uint32_t flags;        /* SRV_FLAG_* */
  uint64_t tick_updates; /* cap on one request's fused-run work per tick, in gate-entry updates
                            (nnz x gates; at least one gate); 0 = no cap.  Keeps ticks short so
                            small requests are not held behind long runs of large ones. */
  uint32_t grid;         /* workgroups of every tick kernel (each walks the tick's work units);
                            0 = 2048, else 1..65536 */
  uint32_t lane_capacity; /* requests whose capacity is at least this many entries run on the
                            large-state lane: the single-state engine (sim_apply_gates, whole
                            circuit, no host round trip per gate) on a stream and host thread of
                            its own, its workspace (sim_workspace_bytes) taken from the pool,
                            concurrently with the batched ticks; queued in a FIFO of their own.
                            0 or SRV_LANE_OFF = no lane (every request batched; the default:
                            server runs with the lane have ended in intermittent GPU memory
                            faults whose cause is not known). */
  uint32_t lane_workers; /* lane threads (each with its own stream), so that as many large
                            requests run at once; 0 = 8, else 1..64 */
  uint32_t max_run_ops;  /* longest fused run a tick takes from one request, in ops (the request's
                            own fuse_max still applies); 0 = 4096.  Long runs on small states are
                            single waves that set a tick's length; cut, they let the other requests
                            of the tick through sooner.  Where runs are cut changes rounding only,
                            and depends on the request and this value alone */
} srv_config;

#define SRV_LANE_OFF 0xFFFFFFFFu

typedef struct srv_stats {
  uint64_t submitted, admitted, completed, failed;
  uint64_t ticks;           /* batched launches */
  uint64_t items;           /* segments executed */
  uint64_t bitslice_runs;   /* fused runs that took the bit-sliced form */
  uint64_t pool_used_bytes, pool_peak_bytes;
  double host_ms;           /* wall time in srv_tick outside the wait for the GPU */
  double wait_ms;           /* wall time srv_tick waited for the GPU */
  double group_ms;          /* of host_ms: grouping fused runs for the bit-sliced form */
  uint64_t lane_completed;  /* requests finished (done or failed) on the large-state lane */
  double lane_ms;           /* wall time the lane spent running requests */
  uint64_t ahead_hits;      /* fused runs whose grouping was made during the previous tick */
  double ahead_ms;          /* of host_ms: work done while a tick ran on the GPU (copying out
                               finished states, grouping expected next runs, compiling queued
                               requests) */
  double copy_ms;           /* copying finished states to host memory, summed over the
                               host threads that did it */
  uint64_t rp_runs;         /* of bitslice_runs: on the register-plane kernel */
  uint64_t paired;          /* branching gates and measurements run in the tick of the fused
                               run before them */
  uint64_t chained;         /* measurements run in the tick of the measurement before them */
} srv_stats;

typedef struct srv_t srv_t;

/* Device bytes one request with this configuration occupies while running;
 * 0 for an invalid configuration. */
size_t srv_footprint(const sim_config* cfg);

/* stream: a hipStream_t, or NULL to let the server create its own (graph
 * capture needs a non-null stream).  pool: device memory of at least
 * budget_bytes, borrowed, or NULL to allocate it.  SIM_E_ARG, SIM_E_NOMEM,
 * SIM_E_HIP. */
int srv_create(const srv_config* cfg, void* stream, void* pool, size_t pool_bytes, srv_t** out);
int srv_destroy(srv_t* s);

/* Queue a request; gates are copied.  *id identifies it.  SIM_E_ARG for an
 * invalid op or configuration (nothing queued), SIM_E_CAPACITY if the
 * footprint exceeds the pool. */
int srv_submit(srv_t* s, const sim_config* cfg, const sim_gate* gates, size_t n, sim_key basis, uint64_t* id);

/* Admit what fits, run one batched tick, retire finished requests.  Writes
 * the numbers of running and queued requests afterwards.  Synchronizes. */
int srv_tick(srv_t* s, uint32_t* running, uint32_t* queued);

/* Tick until nothing is running or queued. */
int srv_run(srv_t* s);

/* State (SRV_*) and, for SRV_FAILED, the error code (SIM_E_CAPACITY when a
 * branching gate would exceed the request's capacity, SIM_E_STATE for a
 * zero-probability measurement). */
int srv_poll(srv_t* s, uint64_t id, int32_t* state, int32_t* error);

/* Copy a finished request's state (storage order), measurement outcomes and
 * counters to caller buffers of cap entries / out_cap outcomes.  *nnz and
 * *n_out receive the sizes; SIM_E_BUFFER if a buffer is too small. */
int srv_result(srv_t* s, uint64_t id, sim_key* keys, sim_c64* amps, uint64_t cap, uint64_t* nnz, int32_t* outcomes,
               uint64_t out_cap, uint64_t* n_out, sim_stats* stats);

/* srv_result into separate arrays, as sim_export_state_soa (key_hi may be
 * NULL); sizes and errors as srv_result. */
int srv_result_soa(srv_t* s, uint64_t id, uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps, uint64_t cap,
                   uint64_t* nnz, int32_t* outcomes, uint64_t out_cap, uint64_t* n_out, sim_stats* stats);

/* Forget a finished or failed request's host-side result. */
int srv_release(srv_t* s, uint64_t id);

int srv_get_stats(srv_t* s, srv_stats* out);
const char* srv_last_error(void);

/* Name of an error code / detail of the last error in this thread. */
const char* sim_strerror(int code);
const char* sim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPARSESIM_H */
