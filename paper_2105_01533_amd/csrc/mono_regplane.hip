// Register-plane fused phase/permutation pass for gfx950 (Sec. 3.2): the
// label bit-planes of a 2048-entry tile stay in VGPRs for the whole run and
// gates address them by index through the GPR indexing mode (see
// regplane_tile.h).  Phases accumulate exactly, as in the bit-sliced form:
// eighth turns in bit-sliced counters, other angles as 64-bit turn fractions,
// one complex multiply per amplitude at the end of the run.
#include <mutex>

#include "regplane_tile.h"

namespace sparsesim {
namespace {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
// The empty asm statement names the highest plane register (rp::kVmax) as
// clobbered, which makes the kernel's VGPR count reach it; the compiler
// itself is held below v80 (amdgpu_num_vgpr), so it never allocates a
// reserved register.
template <bool TURNS>
__global__ __launch_bounds__(64, 2) __attribute__((amdgpu_num_vgpr(40))) void k_mono_rp(
    Buf b, const uint64_t* __restrict__ nnz_p, const RpRec* __restrict__ prog, uint32_t nrec, BsRun run,
    Ctl* ctl) {
  static_assert(rp::kVmax == 230, "the clobber below names the highest plane register");
  asm volatile("" ::: "v230");
  extern __shared__ uint64_t rp_acc[];
  __shared__ uint64_t s_table[32];   // two 16-entry subset-sum tables
  const uint64_t n = *nnz_p;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctl->updates, (unsigned long long)(n * run.n_gates));
    atomicAdd((unsigned long long*)&ctl->mono_updates, (unsigned long long)(n * run.n_gates));
    atomicAdd((unsigned long long*)&ctl->mono_bytes, (unsigned long long)(n * run.bytes_per_entry));
  }
  // One tile per block (the grid covers the largest entry count the host
  // allows for; blocks past the live count do nothing).
  const uint64_t base = (uint64_t)blockIdx.x * 2048;
  if (base >= n) return;
  const uint32_t lim = (uint32_t)(n - base < 2048 ? n - base : 2048);
  rp::rp_tile<TURNS>(b, base, lim, prog, nrec, run, rp_acc, s_table);
}
#pragma clang diagnostic pop

}  // namespace

namespace {

// Register-plane passes of this process never run at the same time on one
// device: waves of two passes with different programs sharing a SIMD gave
// results that depended on the pairing (the GPR-indexed plane accesses),
// while waves of one pass -- one program -- reproduce the LDS-plane pass bit
// for bit.  Each launch records an event on its stream; a launch from another
// stream first waits for it.  (Skipped on a stream under graph capture, where
// the ordering is the graph's.)  The event is made once per device, at
// set-up, so launches allocate nothing.
struct RpOrder {
  std::mutex mu;
  hipEvent_t ev = nullptr;
  hipStream_t last = nullptr;
};

RpOrder& rp_order() {
  static RpOrder orders[64];
  int dev = 0;
  (void)hipGetDevice(&dev);
  return orders[dev & 63];
}

}  // namespace

hipError_t mono_rp_init() {
  RpOrder& o = rp_order();
  std::lock_guard<std::mutex> lk(o.mu);
  if (o.ev) return hipSuccess;
  return hipEventCreateWithFlags(&o.ev, hipEventDisableTiming);
}

void launch_mono_rp(hipStream_t st, Buf b, const uint64_t* nnz, const RpRec* p, uint32_t nrec, const BsRun& run,
                    Ctl* ctl, int grid) {
  RpOrder& o = rp_order();
  std::lock_guard<std::mutex> lk(o.mu);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(st, &cs);
  const bool ordered = cs == hipStreamCaptureStatusNone;
  if (ordered && o.ev && o.last != st) (void)hipStreamWaitEvent(st, o.ev, 0);
  if (run.has_turns)
    hipLaunchKernelGGL(k_mono_rp<true>, dim3(grid), dim3(64), rp::kTurnAccBytes, st, b, nnz, p, nrec, run, ctl);
  else
    hipLaunchKernelGGL(k_mono_rp<false>, dim3(grid), dim3(64), 0, st, b, nnz, p, nrec, run, ctl);
  if (ordered && o.ev && hipEventRecord(o.ev, st) == hipSuccess) o.last = st;
}

}  // namespace sparsesim
