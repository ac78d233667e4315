// Bit-sliced fused phase/permutation pass for gfx950.
//
// A run of phase/permutation gates (Sec. 3.2) is applied to a tile of 2048
// entries per wave: lane l owns entries base + 64*j + l, j = 0..31, and the
// labels are transposed into bit-planes, one 32-bit word per qubit per lane
// (bit j of plane q = qubit q of entry j), held in LDS.  A permutation gate
// on the tile is then one or two bitwise ops on planes:
//     plane[t] ^= AND of the control planes        (X, CNOT, Toffoli, C^nX)
// i.e. 32 entries per lane per instruction, instead of a 128-bit mask test per
// entry.
//
// Phases are accumulated exactly instead of multiplied gate by gate: every
// unit-modulus factor is e^{2 pi i tau} with tau a turn fraction.  Multiples
// of 1/8 turn (Z, S, T, Y and their adjoints) add k to a 3-bit bit-sliced
// counter (three more planes); other angles add tau * 2^64 to a per-entry
// 64-bit turn accumulator, which wraps modulo one turn exactly.  Factors that
// do not depend on the entry (uncontrolled gates' bit-0 factor) are folded
// into run constants by the host.  At the end each amplitude is multiplied
// once by e^{2 pi i (total turns)}; the result differs from gate-by-gate
// multiplication only by rounding (~1e-16 relative per factor).
#include "bitslice_tile.h"

namespace sparsesim {
namespace {

template <bool TURNS>
__global__ __launch_bounds__(64, 2) void k_mono_bs(Buf b, const uint64_t* __restrict__ nnz_p,
                                                const BsGroup* __restrict__ groups, uint32_t ngroups, BsRun run,
                                                Ctl* ctl) {
  extern __shared__ uint32_t lds_all[];
  uint32_t* L = lds_all + threadIdx.x;
  const uint64_t n = *nnz_p;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctl->updates, (unsigned long long)(n * run.n_gates));
    atomicAdd((unsigned long long*)&ctl->mono_updates, (unsigned long long)(n * run.n_gates));
    atomicAdd((unsigned long long*)&ctl->mono_bytes, (unsigned long long)(n * run.bytes_per_entry));
  }
  const uint64_t tiles = (n + 2047) / 2048;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const uint64_t base = tile * 2048;
    const uint32_t lim = (uint32_t)(n - base < 2048 ? n - base : 2048);
    bs::bs_tile<TURNS>(b, base, lim, groups, ngroups, run, L);
  }
}

}  // namespace

void launch_mono_bs(hipStream_t st, Buf b, const uint64_t* nnz, const BsGroup* groups, uint32_t ngroups, const BsRun& run,
                    Ctl* ctl, int grid) {
  // The turn accumulators move into the first 64 planes at the end of a tile.
  const size_t planes = run.has_turns && run.n_planes + kExtraPlanes < 64 ? 64 : run.n_planes + kExtraPlanes;
  const size_t lds = planes * 64 * 4;
  if (run.has_turns)
    hipLaunchKernelGGL(k_mono_bs<true>, dim3(grid), dim3(64), lds, st, b, nnz, groups, ngroups, run, ctl);
  else
    hipLaunchKernelGGL(k_mono_bs<false>, dim3(grid), dim3(64), lds, st, b, nnz, groups, ngroups, run, ctl);
}

}  // namespace sparsesim
