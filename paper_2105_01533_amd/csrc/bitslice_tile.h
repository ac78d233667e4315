// Bit-sliced tile processing shared by the single-state and batched fused
// passes (device code; included by mono_bitslice.hip and batch_kernels.hip).
#pragma once
#include "sim_internal.h"

namespace sparsesim {
namespace bs {


// LSB-first 32x32 bit transpose: out[q] bit j = in[j] bit q (an involution), by
// the recursive block-swap method of Warren, Hacker's Delight, Sec. 7-3: five
// rounds swap 16-, 8-, 4-, 2- and 1-bit blocks between word pairs.
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

// omega_add without branches: k's bits arrive as wave-uniform masks m0, m1,
// m2 (each 0 or ~0).
__device__ __forceinline__ void omega_add_m(uint32_t& e0, uint32_t& e1, uint32_t& e2, uint32_t x, uint32_t m0,
                                            uint32_t m1, uint32_t m2) {
  const uint32_t b0 = x & m0, b1 = x & m1, b2 = x & m2;
  const uint32_t c0 = e0 & b0;
  e0 ^= b0;
  const uint32_t c1 = (e1 & b1) | ((e1 ^ b1) & c0);
  e1 ^= b1 ^ c0;
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

// Turn fractions are read wave-uniformly through the constant address space
// (scalar loads).
typedef const __attribute__((address_space(4))) uint32_t* TauPtr;

// LDS word at byte offset off from the lane's base (L = LDS base + lane).
__device__ __forceinline__ uint32_t& plane(char* Lb, uint32_t off) { return *reinterpret_cast<uint32_t*>(Lb + off); }
__device__ __forceinline__ uint32_t off_t(uint32_t a) { return a & 0xff00u; }
__device__ __forceinline__ uint32_t off_p0(uint32_t a) { return (a >> 8) & 0xff00u; }
__device__ __forceinline__ uint32_t off_p1(uint32_t a) { return (a >> 16) & 0xff00u; }
__device__ __forceinline__ uint32_t off_p2(uint32_t b) { return b & 0xff00u; }

// Flip bodies over N mutually independent ops (all reads, then all writes):
// plane t ^= AND of 0, 1 or 2 control planes.
template <int N>
__device__ __forceinline__ void flip_x(char* Lb, const uint32_t* a) {
  uint32_t tv[N];
#pragma unroll
  for (int u = 0; u < N; ++u) tv[u] = plane(Lb, off_t(a[u]));
#pragma unroll
  for (int u = 0; u < N; ++u) plane(Lb, off_t(a[u])) = ~tv[u];
}
template <int N>
__device__ __forceinline__ void flip_cx(char* Lb, const uint32_t* a) {
  uint32_t tv[N], c0[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    c0[u] = plane(Lb, off_p0(a[u]));
    tv[u] = plane(Lb, off_t(a[u]));
  }
#pragma unroll
  for (int u = 0; u < N; ++u) plane(Lb, off_t(a[u])) = tv[u] ^ c0[u];
}
template <int N>
__device__ __forceinline__ void flip_ccx(char* Lb, const uint32_t* a) {
  uint32_t tv[N], c0[N], c1[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    c0[u] = plane(Lb, off_p0(a[u]));
    c1[u] = plane(Lb, off_p1(a[u]));
    tv[u] = plane(Lb, off_t(a[u]));
  }
#pragma unroll
  for (int u = 0; u < N; ++u) plane(Lb, off_t(a[u])) = tv[u] ^ (c0[u] & c1[u]);
}

// The a words of groups g .. g + 3 of the current batch (a quad).
__device__ __forceinline__ void gather_quad(const uint32_t* a, const uint4& ca, uint32_t g, uint32_t* a16) {
  a16[0] = a[0];
  a16[1] = a[1];
  a16[2] = a[2];
  a16[3] = a[3];
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    a16[4 * k + 0] = (uint32_t)__builtin_amdgcn_readlane(ca.x, g + k);
    a16[4 * k + 1] = (uint32_t)__builtin_amdgcn_readlane(ca.y, g + k);
    a16[4 * k + 2] = (uint32_t)__builtin_amdgcn_readlane(ca.z, g + k);
    a16[4 * k + 3] = (uint32_t)__builtin_amdgcn_readlane(ca.w, g + k);
  }
}

// N eighth-turn ops (all plane reads first), alternating between the two
// counters (e) and (f).
template <int N>
__device__ __forceinline__ void omega_ops(char* Lb, const uint32_t* a, uint32_t& e0, uint32_t& e1, uint32_t& e2,
                                          uint32_t& f0, uint32_t& f1, uint32_t& f2) {
  uint32_t tv[N];
#pragma unroll
  for (int u = 0; u < N; ++u) tv[u] = plane(Lb, off_t(a[u]));
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const uint32_t m0 = (uint32_t)__builtin_amdgcn_sbfe((int)a[u], 2, 1);
    const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)a[u], 3, 1);
    const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int)a[u], 4, 1);
    if (u & 1)
      omega_add_m(f0, f1, f2, tv[u], m0, m1, m2);
    else
      omega_add_m(e0, e1, e2, tv[u], m0, m1, m2);
  }
}

// Apply ngroups grouped ops to the 2048-entry tile at base (lim valid
// entries): labels to LDS planes, gates, labels back, one phase multiply per
// amplitude.  L = LDS base + lane; the all-ones plane must be set.
template <bool TURNS>
__device__ __forceinline__ void bs_tile(const Buf& b, uint64_t base, uint32_t lim, const BsGroup* __restrict__ groups,
                                        uint32_t ngroups, const BsRun& run, uint32_t* L) {
  const int lane = threadIdx.x;
  const int nq = (int)run.n_planes;
    const uint32_t rw = run.words_read | run.words_write;
    if (rw & 3u) load_pair(b.key_lo + base + lane, lim, L, 0, nq);
    __builtin_amdgcn_sched_barrier(0);
    if (rw & 12u) load_pair(b.key_hi + base + lane, lim, L, 2, nq);
    __builtin_amdgcn_sched_barrier(0);
    L[nq * 64] = ~0u;                     // the all-ones plane (the previous tile may have reused it)
    // Eighth-turn counters: OMEGA groups alternate their ops between (e) and
    // (f), two independent dependency chains, summed once at the end.
    uint32_t e0 = 0, e1 = 0, e2 = 0, f0 = 0, f1 = 0, f2 = 0;
    uint64_t turns[TURNS ? 32 : 1];
#pragma unroll
    for (int j = 0; j < (TURNS ? 32 : 1); ++j) turns[j] = 0;
    char* Lb = reinterpret_cast<char*>(L);
    // Groups arrive 64 at a time, one per lane: the a words (and the b words)
    // of a group in one 16-byte vector load, the next batch in flight while
    // this one is used, broadcast with readlane at the group's lane.  A TURN
    // group's turn fractions are read with scalar loads.
    const uint4* gv = reinterpret_cast<const uint4*>(groups);
    const TauPtr taus = (TauPtr)groups;
    uint4 ca = lane < (int)ngroups ? gv[4 * lane] : make_uint4(0, 0, 0, 0);
    uint4 cb = lane < (int)ngroups ? gv[4 * lane + 1] : make_uint4(0, 0, 0, 0);
    // Wait for the first batch here, so that the loops below see it ready.
    asm volatile("" ::"v"(ca.x), "v"(ca.y), "v"(ca.z), "v"(ca.w), "v"(cb.x), "v"(cb.y), "v"(cb.z), "v"(cb.w));
    for (uint32_t g0 = 0; g0 < ngroups; g0 += 64) {
      const bool more = g0 + 64 + lane < ngroups;
      const uint4 na = more ? gv[4 * (g0 + 64 + lane)] : make_uint4(0, 0, 0, 0);
      const uint4 nb = more ? gv[4 * (g0 + 64 + lane) + 1] : make_uint4(0, 0, 0, 0);
      const uint32_t gend = (ngroups - g0 < 64 ? ngroups - g0 : 64);
      uint32_t g = 0;
      while (g < gend) {
        // Groups up to the next TURN group (the turn accumulators stay
        // untouched in this loop).
        for (; g < gend; ++g) {
          uint32_t a[kBsGroup];
          a[0] = __builtin_amdgcn_readlane(ca.x, g);
          a[1] = __builtin_amdgcn_readlane(ca.y, g);
          a[2] = __builtin_amdgcn_readlane(ca.z, g);
          a[3] = __builtin_amdgcn_readlane(ca.w, g);
          const uint32_t shape = bs_shape(a[0]);
          if (shape == kShapeTurn) break;
          // Eight independent flips of one shape when paired with the next
          // group (its a words are at the next lane).
#define BS_FLIP_CASE(SHAPE, BODY)                                  \
  case SHAPE:                                                      \
    if (a[1] & kQuadBit) {                                         \
      uint32_t a16[4 * kBsGroup];                                  \
      gather_quad(a, ca, g, a16);                                  \
      BODY<4 * kBsGroup>(Lb, a16);                                 \
      g += 3;                                                      \
    } else if (a[1] & kPairBit) {                                  \
      uint32_t a8[2 * kBsGroup] = {a[0], a[1], a[2], a[3],         \
                                   (uint32_t)__builtin_amdgcn_readlane(ca.x, g + 1), \
                                   (uint32_t)__builtin_amdgcn_readlane(ca.y, g + 1), \
                                   (uint32_t)__builtin_amdgcn_readlane(ca.z, g + 1), \
                                   (uint32_t)__builtin_amdgcn_readlane(ca.w, g + 1)}; \
      BODY<2 * kBsGroup>(Lb, a8);                                  \
      ++g;                                                         \
    } else {                                                       \
      BODY<kBsGroup>(Lb, a);                                       \
    }                                                              \
    continue;
          switch (shape) {
            BS_FLIP_CASE(kShapeX, flip_x)
            BS_FLIP_CASE(kShapeCX, flip_cx)
            BS_FLIP_CASE(kShapeCCX, flip_ccx)
            default:
              break;
          }
#undef BS_FLIP_CASE
          if (shape == kShapeOmega) {
            // Eighth-turn phase ops conditioned on their target bit only
            // (Z, S, T and their adjoints): read-only on the planes.
            if (a[1] & kQuadBit) {
              uint32_t a16[4 * kBsGroup];
              gather_quad(a, ca, g, a16);
              omega_ops<4 * kBsGroup>(Lb, a16, e0, e1, e2, f0, f1, f2);
              g += 3;
            } else if (a[1] & kPairBit) {
              uint32_t a8[2 * kBsGroup] = {a[0], a[1], a[2], a[3],
                                           (uint32_t)__builtin_amdgcn_readlane(ca.x, g + 1),
                                           (uint32_t)__builtin_amdgcn_readlane(ca.y, g + 1),
                                           (uint32_t)__builtin_amdgcn_readlane(ca.z, g + 1),
                                           (uint32_t)__builtin_amdgcn_readlane(ca.w, g + 1)};
              omega_ops<2 * kBsGroup>(Lb, a8, e0, e1, e2, f0, f1, f2);
              ++g;
            } else {
              omega_ops<kBsGroup>(Lb, a, e0, e1, e2, f0, f1, f2);
            }
          } else {
            // General group: every op writes its plane t; a flip xors the
            // condition in, an eighth-turn phase op's t is a fourth condition
            // plane (its target bit, or the all-ones plane) and is written
            // back unchanged.
            uint32_t bw[kBsGroup];
            bw[0] = __builtin_amdgcn_readlane(cb.x, g);
            bw[1] = __builtin_amdgcn_readlane(cb.y, g);
            bw[2] = __builtin_amdgcn_readlane(cb.z, g);
            bw[3] = __builtin_amdgcn_readlane(cb.w, g);
            uint32_t c0[kBsGroup], c1[kBsGroup], c2[kBsGroup], tv[kBsGroup];
#pragma unroll
            for (int u = 0; u < kBsGroup; ++u) {
              c0[u] = plane(Lb, off_p0(a[u]));
              c1[u] = plane(Lb, off_p1(a[u]));
              c2[u] = plane(Lb, off_p2(bw[u]));
              tv[u] = plane(Lb, off_t(a[u]));
            }
            __builtin_amdgcn_sched_barrier(0);
            uint32_t cond[kBsGroup];
#pragma unroll
            for (int u = 0; u < kBsGroup; ++u) {
              cond[u] = c0[u] & c1[u] & c2[u];
              const uint32_t fm = (a[u] & 3u) == kBsFlip ? ~0u : 0u;
              plane(Lb, off_t(a[u])) = tv[u] ^ (cond[u] & fm);
            }
            if (shape == kShapePhase) {
#pragma unroll
              for (int u = 0; u < kBsGroup; ++u)
                if ((a[u] & 3u) == kBsOmega) omega_add(e0, e1, e2, cond[u] & tv[u], (a[u] >> 2) & 7u);
            }
          }
        }
        if (g >= gend) break;
        // A TURN group: four turn ops (read-only on the planes).
        if (TURNS) {
          uint32_t a[kBsGroup], bw[kBsGroup];
          a[0] = __builtin_amdgcn_readlane(ca.x, g);
          a[1] = __builtin_amdgcn_readlane(ca.y, g);
          a[2] = __builtin_amdgcn_readlane(ca.z, g);
          a[3] = __builtin_amdgcn_readlane(ca.w, g);
          bw[0] = __builtin_amdgcn_readlane(cb.x, g);
          bw[1] = __builtin_amdgcn_readlane(cb.y, g);
          bw[2] = __builtin_amdgcn_readlane(cb.z, g);
          bw[3] = __builtin_amdgcn_readlane(cb.w, g);
          // The group's turn fractions: scalar loads, issued before the plane
          // reads so that their latency overlaps the reads and transposes.
          const uint32_t tg = 16u * (g0 + g) + 8u;   // in 32-bit words
          uint64_t tau[kBsGroup];
#pragma unroll
          for (int u = 0; u < kBsGroup; ++u) tau[u] = ((uint64_t)taus[tg + 2 * u + 1] << 32) | taus[tg + 2 * u];
          uint32_t x[kBsGroup];
          if (a[1] & kBareBit) {
#pragma unroll
            for (int u = 0; u < kBsGroup; ++u) x[u] = plane(Lb, off_t(a[u]));
          } else {
#pragma unroll
            for (int u = 0; u < kBsGroup; ++u)
              x[u] = plane(Lb, off_p0(a[u])) & plane(Lb, off_p1(a[u])) & plane(Lb, off_p2(bw[u])) &
                     plane(Lb, off_t(a[u]));
          }
          // Entry j's table offset, 8 x (the ops, bit u = op u, whose
          // condition holds for it), is byte j >> 3 of B[j & 7]: bit j of mask
          // u moves to bit 8 (j >> 3) + 3 + u by one constant shift, and the
          // four masks merge under disjoint byte-lane masks.
          uint32_t B[8];
#pragma unroll
          for (int w = 0; w < 8; ++w) {
            uint32_t r = 0;
#pragma unroll
            for (int u = 0; u < kBsGroup; ++u) {
              const int sh = w - 3 - u;
              const uint32_t y = sh >= 0 ? x[u] >> sh : x[u] << -sh;
              r |= y & (0x01010101u << (3 + u));
            }
            B[w] = r;
            // Keep the byte extraction below a single bit-field extract per
            // entry (otherwise it is folded back into shifts and masks).
            asm volatile("" : "+v"(B[w]));
          }
          // An entry gains the sum of the fractions of the ops whose condition
          // holds for it: one of 16 subset sums, kept as 8-byte words in a
          // static LDS table (entry m = the sum over the ops named by m's
          // bits) and read per entry with one 64-bit LDS load.  Its address
          // is a constant, so an entry's load address is its index times
          // eight.  The wave's LDS accesses complete in order, so the table is
          // written before any load of it.
          __shared__ uint64_t s_table[16];
          uint64_t S = 0;
#pragma unroll
          for (int u = 0; u < kBsGroup; ++u) S += tau[u] & (0ull - (uint64_t)((lane >> u) & 1));
          // Every lane forms S, so the loads are not moved into the branch.
          asm volatile("" ::"v"(S));
          const char* table = reinterpret_cast<const char*>(s_table);
          if (lane < 16) s_table[lane] = S;
          // Table loads go out fourteen at a time (the LDS counter counts to
          // fifteen) before their sums are added.
#pragma unroll
          for (int j0 = 0; j0 < 32; j0 += 14) {
            uint64_t v[14];
#pragma unroll
            for (int k = 0; k < 14 && j0 + k < 32; ++k) {
              const int j = j0 + k;
              const uint32_t off = __builtin_amdgcn_ubfe(B[j & 7], 8 * (j >> 3), 8);
              v[k] = *reinterpret_cast<const uint64_t*>(table + off);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 14 && j0 + k < 32; ++k) turns[j0 + k] += v[k];
          }
        }
        ++g;
      }
      ca = na;
      cb = nb;
    }
    {
      // (e) += (f), bit-sliced, modulo 8.
      const uint32_t c0 = e0 & f0;
      e0 ^= f0;
      const uint32_t c1 = (e1 & f1) | ((e1 ^ f1) & c0);
      e1 ^= f1 ^ c0;
      e2 ^= f2 ^ c1;
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
