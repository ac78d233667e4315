// A branching gate on a small state in one block, with the partner index in
// LDS (Sec. 3.1): shared by the single-state kernel (sim_kernels.hip) and
// the batched tick (batch_kernels.hip).  Device code only.
//
// The same entries are indexed as by the global index (under the controls,
// pivot bit clear), by the same label hash; the same look-ups (label ^ x from
// the pivot-set entries) pair them; Eq. 2 is evaluated by ent::u2_eval and the
// outputs are written in entry order.  The outputs and their order are
// therefore those of the index-build / probe / write kernels, in one launch
// and with no global index to fill, probe or empty.  A slot holds an 18-bit
// fingerprint above entry index + 1 (kIdxBits = 14 bits; 0 = empty); the table has twice
// as many slots as the largest state, so it is at most half full and every
// probe sequence meets an empty slot.
#pragma once
#include "entry_ops.h"

namespace sparsesim {
namespace lds {

constexpr uint32_t kSlots = 2 * kLdsU2Max;
constexpr int kThreads = 1024;
constexpr int kItems = (int)(kLdsU2Max / kThreads);
constexpr int kWaves = kThreads / 64;
constexpr int kIdxBits = 14;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
static_assert(kLdsU2Max < (1u << kIdxBits) && kItems * kThreads == (int)kLdsU2Max, "index field of a slot");

// LDS of one block (about 96 KB); declared by the kernel, whatever the label
// width, so that both widths share it.
struct Smem {
  uint32_t tab[kSlots];
  uint32_t par[kLdsU2Max];
  uint32_t wave[kWaves];
  uint32_t red_u[kWaves];
  double red_d[kWaves];
};

struct Totals {
  uint32_t out;       // outputs (entries of the new state)
  uint32_t dropped;   // outputs T_eps dropped
  double mass;        // their |a|^2, summed in a fixed order
  uint32_t ix[4];     // index work: inserts, CAS attempts, look-ups, slots read by look-ups
};

// Exclusive prefix over the block of e in {0, 1, 2}, in thread order; *total
// gets the block's sum.  Every thread calls it.
__device__ __forceinline__ uint32_t prefix012(uint32_t e, Smem& sm, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t b1 = __ballot(e >= 1), b2 = __ballot(e >= 2);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t pre = __popcll(b1 & lt) + __popcll(b2 & lt);
  if (lane == 0) sm.wave[wid] = __popcll(b1) + __popcll(b2);
  __syncthreads();
  uint32_t woff = 0, tot = 0;
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t x = sm.wave[w];
    woff += w < wid ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return woff + pre;
}

// Block sums in a fixed order: a butterfly in each wave, then the waves in
// order.  Every thread calls them and gets the sum.
__device__ __forceinline__ uint32_t sum_u(uint32_t v, Smem& sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sm.red_u[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
  for (int w = 0; w < kWaves; ++w) r += sm.red_u[w];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double sum_d(double v, Smem& sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sm.red_d[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sm.red_d[0];
  for (int w = 1; w < kWaves; ++w) r += sm.red_d[w];
  __syncthreads();
  return r;
}

// The gate on entries [0, n) of `in` (n <= kLdsU2Max, blockDim.x ==
// kThreads), written to `out` (which holds cap entries).
template <bool WIDE>
__device__ Totals u2_block(const Buf& in, const Buf& out, uint32_t n, const U2Desc& d, uint64_t cap, Smem& sm) {
  constexpr uint32_t kMask = kSlots - 1;
  for (uint32_t k = threadIdx.x; k < kSlots; k += kThreads) sm.tab[k] = 0u;
  uint32_t inserts = 0, cas = 0, lookups = 0, steps = 0;
  uint64_t lo[kItems], hi[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = (uint32_t)k * kThreads + threadIdx.x;
    lo[k] = hi[k] = 0;
    if (i < n) {
      lo[k] = in.key_lo[i];
      hi[k] = WIDE ? in.key_hi[i] : 0ull;
      sm.par[i] = kNoPartner;
    }
  }
  __syncthreads();
  // Index the pivot-clear entries under the controls.
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = (uint32_t)k * kThreads + threadIdx.x;
    if (i >= n || !ent::ctrl_ok(d, lo[k], hi[k], WIDE) || ent::pivot_set(d, lo[k], hi[k], WIDE)) continue;
    const uint64_t h = ent::hash_label(lo[k], hi[k]);
    const uint32_t val = ((uint32_t)(h >> (32 + kIdxBits)) << kIdxBits) | (i + 1u);
    uint32_t slot = (uint32_t)h & kMask;
    ++inserts;
    for (uint32_t p = 0; p < kSlots; ++p) {
      ++cas;
      if (atomicCAS(&sm.tab[slot], 0u, val) == 0u) break;
      slot = (slot + 1u) & kMask;
    }
  }
  __syncthreads();
  // Each pivot-set entry under the controls looks up label ^ x; a hit makes
  // the two entries each other's partner (a pivot-clear entry has at most one).
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = (uint32_t)k * kThreads + threadIdx.x;
    if (i >= n || !ent::ctrl_ok(d, lo[k], hi[k], WIDE) || !ent::pivot_set(d, lo[k], hi[k], WIDE)) continue;
    const uint64_t qlo = lo[k] ^ d.x_lo, qhi = WIDE ? (hi[k] ^ d.x_hi) : 0ull;
    const uint64_t h = ent::hash_label(qlo, qhi);
    const uint32_t fp = (uint32_t)(h >> (32 + kIdxBits));
    uint32_t slot = (uint32_t)h & kMask;
    ++lookups;
    for (uint32_t p = 0; p < kSlots; ++p) {
      const uint32_t v = sm.tab[slot];
      ++steps;
      if (v == 0u) break;
      if ((v >> kIdxBits) == fp) {
        const uint32_t j = (v & kIdxMask) - 1u;
        if (in.key_lo[j] == qlo && (!WIDE || in.key_hi[j] == qhi)) {
          sm.par[i] = j;
          sm.par[j] = i;
          break;
        }
      }
      slot = (slot + 1u) & kMask;
    }
  }
  __syncthreads();
  // Evaluate and write in entry order, kThreads entries per round.  A
  // position at or past cap is not written: the gate then overflows (the
  // caller sees out > cap) and `out`, the state's other buffer, holds nothing
  // the state needs.
  uint32_t run = 0, dropped = 0;
  double mass = 0.0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if ((uint32_t)k * kThreads >= n) break;   // uniform: no entry in this round or later ones
    const uint32_t i = (uint32_t)k * kThreads + threadIdx.x;
    ent::U2Out r;
    r.mode = 2;
    r.o0 = r.o1 = make_double2(0.0, 0.0);
    bool k0 = false, k1 = false;
    if (i < n) {
      r = ent::u2_eval(d, WIDE, in.amp, lo[k], hi[k], in.amp[i], sm.par[i]);
      if (r.mode == 0) {
        k0 = ent::survives(r.o0, d.eps);
        dropped += k0 ? 0u : 1u;
        mass += ent::dropped_mass(r.o0, k0);
      } else if (r.mode == 1) {
        k0 = ent::survives(r.o0, d.eps);
        k1 = ent::survives(r.o1, d.eps);
        dropped += (k0 ? 0u : 1u) + (k1 ? 0u : 1u);
        mass += ent::dropped_mass(r.o0, k0) + ent::dropped_mass(r.o1, k1);
      }
    }
    uint32_t tt;
    uint64_t p = run + prefix012((k0 ? 1u : 0u) + (k1 ? 1u : 0u), sm, &tt);
    run += tt;
    if (r.mode == 0) {
      if (k0 && p < cap) {
        out.key_lo[p] = lo[k];
        if (WIDE) out.key_hi[p] = hi[k];
        out.amp[p] = r.o0;
      }
    } else if (r.mode == 1) {
      const bool v = ent::pivot_set(d, lo[k], hi[k], WIDE);
      const uint64_t lo0 = v ? lo[k] ^ d.x_lo : lo[k], hi0 = v ? hi[k] ^ d.x_hi : hi[k];
      if (k0) {
        if (p < cap) {
          out.key_lo[p] = lo0;
          if (WIDE) out.key_hi[p] = hi0;
          out.amp[p] = r.o0;
        }
        ++p;
      }
      if (k1 && p < cap) {
        out.key_lo[p] = lo0 ^ d.x_lo;
        if (WIDE) out.key_hi[p] = hi0 ^ d.x_hi;
        out.amp[p] = r.o1;
      }
    }
  }
  Totals t;
  t.out = run;
  t.dropped = sum_u(dropped, sm);
  t.mass = sum_d(mass, sm);
  t.ix[0] = sum_u(inserts, sm);
  t.ix[1] = sum_u(cas, sm);
  t.ix[2] = sum_u(lookups, sm);
  t.ix[3] = sum_u(steps, sm);
  return t;
}

}  // namespace lds
}  // namespace sparsesim
