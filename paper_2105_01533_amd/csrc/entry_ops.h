// Per-entry arithmetic shared by the single-state kernels (sim_kernels.hip)
// and the batched kernels (batch_kernels.hip), so that both families compute
// the same values: complex products with a fixed order of operations, the
// prune test T_eps, the label hash of the partner index, and Eq. 2 on one
// entry with the pair rule of Sec. 3.1.  Device code only.
#pragma once
#include "sim_internal.h"

namespace sparsesim {
namespace ent {

// (a.re b.re - a.im b.im, a.re b.im + a.im b.re); the library is built with
// -ffp-contract=off, so no step is fused.
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
// c ? x : y component by component (a conditional on the vector type itself
// is lowered through a stack temporary).
__device__ __forceinline__ double2 sel2(bool c, double2 x, double2 y) {
  return make_double2(c ? x.x : y.x, c ? x.y : y.y);
}

// T_eps: an entry survives iff re*re + im*im >= eps and it is not exactly
// zero (strict < drops).
__device__ __forceinline__ bool survives(double2 a, double eps) {
  return !((a.x * a.x + a.y * a.y < eps) || (a.x == 0.0 && a.y == 0.0));
}

// 64-bit finalizer of MurmurHash3 (Appleby), applied to a 128-bit label.
__device__ __forceinline__ uint64_t hash_label(uint64_t lo, uint64_t hi) {
  uint64_t k = lo + hi * 0x9E3779B97F4A7C15ull;
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ bool ctrl_ok(const U2Desc& d, uint64_t lo, uint64_t hi, bool wide) {
  return (lo & d.ctrl_lo) == d.ctrl_lo && (!wide || (hi & d.ctrl_hi) == d.ctrl_hi);
}

__device__ __forceinline__ bool pivot_set(const U2Desc& d, uint64_t lo, uint64_t hi, bool wide) {
  const uint64_t w = (wide && d.target >= 64) ? hi : lo;
  return ((w >> (d.target & 63)) & 1ull) != 0;
}

// Branching gate outputs of one entry (label lo/hi, amplitude a), given the
// index j of its partner label ^ x in the same buffer (amp) or kNoPartner:
// Eq. 2 with the pair rule (of two present partners the one with the pivot
// bit set emits).  mode 0: the label is outside the controls and passes
// through (o0 = a); 1: it emits the pair, o0 for b0 (pivot bit clear) and
// o1 for b0 ^ x; 2: its partner emits, nothing here.
struct U2Out {
  int mode;
  double2 o0, o1;
};
__device__ __forceinline__ U2Out u2_eval(const U2Desc& d, bool wide, const double2* __restrict__ amp, uint64_t lo,
                                         uint64_t hi, double2 a, uint32_t j) {
  U2Out r;
  r.o0 = a;   // every path writes both outputs (keeps them in registers)
  r.o1 = a;
  if (!ctrl_ok(d, lo, hi, wide)) {
    r.mode = 0;
    return r;
  }
  const bool v = pivot_set(d, lo, hi, wide);
  if (!v && j != kNoPartner) {
    r.mode = 2;
    return r;
  }
  const double2 zero = make_double2(0.0, 0.0);
  double2 aj = zero;
  if (v && j != kNoPartner) aj = amp[j];
  const double2 a0 = sel2(v, aj, a);
  const double2 a1 = sel2(v, a, zero);
  // The off-diagonal sign comes from b0, the pair's label with the pivot clear.
  const uint64_t b0lo = v ? lo ^ d.x_lo : lo, b0hi = v ? hi ^ d.x_hi : hi;
  const bool odd = ((__popcll(b0lo & d.z_lo) + (wide ? __popcll(b0hi & d.z_hi) : 0)) & 1) != 0;
  double2 p01 = cmul(d.u[1], a1), p10 = cmul(d.u[2], a0);
  if (odd) {
    p01 = make_double2(-p01.x, -p01.y);
    p10 = make_double2(-p10.x, -p10.y);
  }
  r.mode = 1;
  r.o0 = cadd(cmul(d.u[0], a0), p01);
  r.o1 = cadd(p10, cmul(d.u[3], a1));
  return r;
}

// |a|^2 of an output that T_eps drops (0 for exact zeros), for the pruned
// mass counter.
__device__ __forceinline__ double dropped_mass(double2 a, bool kept) { return kept ? 0.0 : a.x * a.x + a.y * a.y; }

}  // namespace ent
}  // namespace sparsesim
