// Register-plane fused phase/permutation pass for gfx950 (Sec. 3.2): the
// label bit-planes of a 2048-entry tile stay in VGPRs for the whole run and
// gates address them by index through the GPR indexing mode (see
// regplane_tile.h).  Phases accumulate exactly, as in the bit-sliced form:
// eighth turns in bit-sliced counters, other angles as 64-bit turn fractions,
// one complex multiply per amplitude at the end of the run.
#include "regplane_tile.h"

namespace sparsesim {
namespace {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
// VMAX: the highest plane register of the variant.  The empty asm statement
// names it as clobbered, which makes the kernel's VGPR count reach it; the
// compiler itself is held below v80 (amdgpu_num_vgpr), so it never allocates
// a reserved register.
template <bool TURNS, uint32_t VMAX>
__global__ __launch_bounds__(64, 2) __attribute__((amdgpu_num_vgpr(40))) void k_mono_rp(
    Buf b, const uint64_t* __restrict__ nnz_p, const RpRec* __restrict__ prog, uint32_t nrec, BsRun run,
    Ctl* ctl) {
  if constexpr (VMAX == rp::kVmaxSmall) asm volatile("" ::: "v131");
  else if constexpr (VMAX == rp::kVmaxMid) asm volatile("" ::: "v163");
  else asm volatile("" ::: "v230");
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

template <bool TURNS>
void launch_variant(hipStream_t st, Buf b, const uint64_t* nnz, const RpRec* prog, uint32_t nrec,
                    const BsRun& run, Ctl* ctl, int grid) {
  const size_t lds = TURNS ? rp::kTurnAccBytes : 0;
  const uint32_t planes = run.n_planes + 3;   // labels, all-ones, scratch, zero
  if (planes <= 32)
    hipLaunchKernelGGL((k_mono_rp<TURNS, rp::kVmaxSmall>), dim3(grid), dim3(64), lds, st, b, nnz, prog, nrec, run,
                       ctl);
  else if (planes <= 64)
    hipLaunchKernelGGL((k_mono_rp<TURNS, rp::kVmaxMid>), dim3(grid), dim3(64), lds, st, b, nnz, prog, nrec, run, ctl);
  else
    hipLaunchKernelGGL((k_mono_rp<TURNS, rp::kVmaxWide>), dim3(grid), dim3(64), lds, st, b, nnz, prog, nrec, run,
                       ctl);
}

}  // namespace

void launch_mono_rp(hipStream_t st, Buf b, const uint64_t* nnz, const RpRec* p, uint32_t nrec, const BsRun& run,
                    Ctl* ctl, int grid) {
  if (run.has_turns)
    launch_variant<true>(st, b, nnz, p, nrec, run, ctl, grid);
  else
    launch_variant<false>(st, b, nnz, p, nrec, run, ctl, grid);
}

}  // namespace sparsesim
