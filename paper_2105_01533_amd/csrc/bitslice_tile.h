// Bit-sliced tile processing shared by the single-state and batched fused
// passes (device code; included by mono_bitslice.hip and batch_kernels.hip).
#pragma once
#include "sim_internal.h"

namespace sparsesim {
namespace bs {


// LSB-first 32x32 bit transpose: out[q] bit j = in[j] bit q (an involution).
__device__ __forceinline__ void transpose32(uint32_t (&A)[32]) {
  uint32_t m = 0x0000FFFFu;
#pragma unroll
  for (int j = 16; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
    for (int k = 0; k < 32; k = (k + j + 1) & ~j) {
      const uint32_t t = ((A[k] >> j) ^ A[k + j]) & m;
      A[k] ^= t << j;
      A[k + j] ^= t;
    }
  }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Add the constant k (0..7) to the bit-sliced counter (e2 e1 e0) where x is set.
__device__ __forceinline__ void omega_add(uint32_t& e0, uint32_t& e1, uint32_t& e2, uint32_t x, uint32_t k) {
  const uint32_t b0 = (k & 1u) ? x : 0u, b1 = (k & 2u) ? x : 0u, b2 = (k & 4u) ? x : 0u;
  const uint32_t c0 = e0 & b0;
  e0 ^= b0;
  const uint32_t s1 = e1 ^ b1;
  const uint32_t c1 = (e1 & b1) | (s1 & c0);
  e1 = s1 ^ c0;
  e2 ^= b2 ^ c1;
}

// Load the lane's 32 labels' 64-bit word (src already offset by base + lane;
// entry j at src[64 j]) and transpose both 32-bit halves into planes
// 32*w0 .. 32*w0+63 of LDS.
__device__ __forceinline__ void load_pair(const uint64_t* __restrict__ src, uint32_t lim, uint32_t* L, int w0,
                                          int nq) {
  const int lane = threadIdx.x;
  uint32_t a[32], c[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const uint64_t v = (64u * j + lane < lim) ? src[64 * j] : 0ull;
    a[j] = (uint32_t)v;
    c[j] = (uint32_t)(v >> 32);
  }
  transpose32(a);
  transpose32(c);
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    if (32 * w0 + q < nq) L[(32 * w0 + q) * 64] = a[q];
    if (32 * w0 + 32 + q < nq) L[(32 * w0 + 32 + q) * 64] = c[q];
  }
}

// Planes 32*w0 .. +63 back to the lane's 64-bit label words.
__device__ __forceinline__ void store_pair(uint64_t* __restrict__ dst, uint32_t lim, const uint32_t* L, int w0,
                                           int nq) {
  const int lane = threadIdx.x;
  uint32_t a[32], c[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    a[q] = 32 * w0 + q < nq ? L[(32 * w0 + q) * 64] : 0u;
    c[q] = 32 * w0 + 32 + q < nq ? L[(32 * w0 + 32 + q) * 64] : 0u;
  }
  transpose32(a);
  transpose32(c);
#pragma unroll
  for (int j = 0; j < 32; ++j)
    if (64u * j + lane < lim) dst[64 * j] = ((uint64_t)c[j] << 32) | a[j];
}

// omega^k = e^{i pi k / 4}, exact: (1,0) or (h,h) rotated by i^(k >> 1).
__device__ __forceinline__ double2 omega_pow(uint32_t k) {
  const double h = 0.70710678118654752440;
  const double x = (k & 1u) ? h : 1.0, y = (k & 1u) ? h : 0.0;
  const uint32_t r = (k >> 1) & 3u;
  const double re = r == 0 ? x : (r == 1 ? -y : (r == 2 ? -x : y));
  const double im = r == 0 ? y : (r == 1 ? x : (r == 2 ? -y : -x));
  return make_double2(re, im);
}

// One op of a group: fields broadcast from the lane that loaded it.
struct OpS {
  uint32_t op, t, p0, p1, p2, k;
  uint64_t tau;
};

__device__ __forceinline__ OpS op_from_lane(const uint4& v, int src) {
  const uint32_t x = __builtin_amdgcn_readlane(v.x, src);
  const uint32_t y = __builtin_amdgcn_readlane(v.y, src);
  const uint32_t z = __builtin_amdgcn_readlane(v.z, src);
  const uint32_t w = __builtin_amdgcn_readlane(v.w, src);
  OpS o;
  o.op = x & 0xffu;
  o.t = ((x >> 8) & 0xffu) * 64u;
  o.p0 = ((x >> 16) & 0xffu) * 64u;
  o.p1 = (x >> 24) * 64u;
  o.p2 = (y & 0xffu) * 64u;
  o.k = (y >> 8) & 0xffu;
  o.tau = ((uint64_t)w << 32) | z;
  return o;
}

// Ops arrive 64 at a time, one per lane (one vector load per 64 ops, the next
// batch in flight while the current one is used); each group of kBsGroup ops
// is broadcast with readlane, all its plane reads are issued, then it computes
// and writes.  The LDS holds nq label planes, an all-ones plane (index nq) that
// unused condition slots name, and a scratch plane (nq + 1) for padding ops.
// Apply ngroups grouped ops to the 2048-entry tile at base (lim valid
// entries): labels to LDS planes, gates, labels back, one phase multiply per
// amplitude.  L = LDS base + lane; the all-ones plane must be set.
template <bool TURNS>
__device__ __forceinline__ void bs_tile(const Buf& b, uint64_t base, uint32_t lim, const BsOpG* __restrict__ ops,
                                        uint32_t ngroups, const BsRun& run, uint32_t* L) {
  const int lane = threadIdx.x;
  const int nq = (int)run.n_planes;
  const uint4* opv = reinterpret_cast<const uint4*>(ops);
  const uint32_t nops = ngroups * kBsGroup;
    const uint32_t rw = run.words_read | run.words_write;
    if (rw & 3u) load_pair(b.key_lo + base + lane, lim, L, 0, nq);
    __builtin_amdgcn_sched_barrier(0);
    if (rw & 12u) load_pair(b.key_hi + base + lane, lim, L, 2, nq);
    __builtin_amdgcn_sched_barrier(0);
    L[nq * 64] = ~0u;                     // the all-ones plane (the previous tile may have reused it)
    uint32_t e0 = 0, e1 = 0, e2 = 0;
    uint64_t turns[TURNS ? 32 : 1];
#pragma unroll
    for (int j = 0; j < (TURNS ? 32 : 1); ++j) turns[j] = 0;
    uint4 cur = lane < (int)nops ? opv[lane] : make_uint4(0, 0, 0, 0);
    for (uint32_t b0 = 0; b0 < nops; b0 += 64) {
      const uint4 nxt = b0 + 64 + lane < nops ? opv[b0 + 64 + lane] : make_uint4(0, 0, 0, 0);
      const uint32_t gend = (nops - b0 < 64 ? nops - b0 : 64);
      for (uint32_t g = 0; g < gend; g += kBsGroup) {
        OpS o[kBsGroup];
        uint32_t cond[kBsGroup], tv[kBsGroup];
#pragma unroll
        for (int u = 0; u < kBsGroup; ++u) o[u] = op_from_lane(cur, g + u);
#pragma unroll
        for (int u = 0; u < kBsGroup; ++u) {
          cond[u] = L[o[u].p0] & L[o[u].p1] & L[o[u].p2];
          tv[u] = L[o[u].t];
        }
        // Every op writes its plane t: a flip xors the condition in; a phase
        // op's t is a fourth condition plane (its target bit, or the all-ones
        // plane) and is written back unchanged.
#pragma unroll
        for (int u = 0; u < kBsGroup; ++u) L[o[u].t] = tv[u] ^ (o[u].op == kBsFlip ? cond[u] : 0u);
#pragma unroll
        for (int u = 0; u < kBsGroup; ++u) {
          const uint32_t x = cond[u] & tv[u];
          if (o[u].op == kBsFlip) {
          } else if (o[u].op == kBsOmega) {
            omega_add(e0, e1, e2, x, o[u].k);
          } else if (TURNS) {
            const uint32_t tlo = (uint32_t)o[u].tau, thi = (uint32_t)(o[u].tau >> 32);
#pragma unroll
            for (int j = 0; j < 32; ++j) {
              const uint32_t m = (uint32_t)(-(int32_t)((x >> j) & 1u));
              turns[j] += ((uint64_t)(thi & m) << 32) | (tlo & m);
            }
          }
        }
      }
      cur = nxt;
    }
    // Labels back to memory (only words some gate flips).
    __builtin_amdgcn_sched_barrier(0);
    if (run.words_write & 3u) store_pair(b.key_lo + base + lane, lim, L, 0, nq);
    __builtin_amdgcn_sched_barrier(0);
    if (run.words_write & 12u) store_pair(b.key_hi + base + lane, lim, L, 2, nq);
    __builtin_amdgcn_sched_barrier(0);
    // One complex multiply per amplitude by the accumulated phase.  The label
    // planes are dead now: the turn accumulators move to LDS (two words per
    // entry per lane) so the loop below need not be unrolled.
    if (run.has_phase) {
      if (TURNS) {
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          L[(2 * j) * 64] = (uint32_t)turns[j];
          L[(2 * j + 1) * 64] = (uint32_t)(turns[j] >> 32);
        }
      }
      double2* amp = b.amp + base + lane;
#pragma unroll 1
      for (int j = 0; j < 32; ++j) {
        if (64u * j + lane >= lim) break;
        const uint32_t k = ((((e2 >> j) & 1u) << 2) | (((e1 >> j) & 1u) << 1) | ((e0 >> j) & 1u)) + run.g_omega;
        double2 f;
        if (!TURNS && run.g_turn == 0) {
          f = omega_pow(k);
        } else {
          const uint64_t tj = TURNS ? (((uint64_t)L[(2 * j + 1) * 64] << 32) | L[(2 * j) * 64]) : 0ull;
          const uint64_t T = tj + run.g_turn + ((uint64_t)(k & 7u) << 61);
          double sn, cs;
          sincospi((double)(T >> 11) * 0x1p-52, &sn, &cs);   // angle = 2 pi T / 2^64
          f = make_double2(cs, sn);
        }
        amp[64 * j] = cmul(amp[64 * j], f);
      }
    }
}

}  // namespace bs
}  // namespace sparsesim
