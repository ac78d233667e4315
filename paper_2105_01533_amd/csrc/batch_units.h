// Work-unit lookup shared by the batched kernels.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace sparsesim {

// Largest i in [0, n) with u0[i] <= u (u0 ascending, u0[0] = 0).
__device__ __forceinline__ int find_item(const uint32_t* __restrict__ u0, int n, uint32_t u) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (u0[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace sparsesim
