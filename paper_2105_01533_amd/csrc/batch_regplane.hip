// Batched fused runs on the register-plane tile: every unit (kChunk entries of
// one state) whose item carries a register-plane program is one tile.  Built
// in a translation unit of its own, without machine loop-invariant code
// motion: hoisting the phase epilogue's constants out of the loop over units
// would keep them live across the tile, whose compiler code must fit below
// the planes' registers.
#include "batch_units.h"
#include "regplane_tile.h"

namespace sparsesim {
namespace {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__global__ __launch_bounds__(64, 2) __attribute__((amdgpu_num_vgpr(40))) void kb_mono(
    const BTick* __restrict__ hdr, const BItem* __restrict__ items, const uint32_t* __restrict__ units) {
  asm volatile("" ::: "v230");
  extern __shared__ uint64_t rp_acc[];
  __shared__ uint64_t s_table[32];
  const int n = (int)hdr->n_mono;
  if (n == 0) return;
  const uint32_t* u0 = units + hdr->mono_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = items[i];
    if (!it.prog) continue;   // the per-entry kernel's
    const uint64_t base = (uint64_t)(u - u0[i]) * kChunk;
    const uint32_t lim = (uint32_t)(it.nnz - base < kChunk ? it.nnz - base : kChunk);
    rp::rp_tile<true>(it.in, base, lim, it.prog, it.nrec, it.run, rp_acc, s_table);
  }
}
#pragma clang diagnostic pop

}  // namespace

void launch_batch_mono_rp(hipStream_t st, const BTick* hdr, const BItem* items, const uint32_t* units, int grid) {
  hipLaunchKernelGGL(kb_mono, dim3(grid), dim3(64), rp::kTurnAccBytes, st, hdr, items, units);
}

}  // namespace sparsesim
