// Batched kernels: one tick applies one segment to every active state.
//
// Every kernel runs a fixed grid (so the whole tick can be captured once as a
// hipGraph and replayed) and walks a flat list of work units; unit u belongs
// to the item whose first-unit entry is the largest one <= u.  Units are
// kChunk entries of one state (kFillUnit slots for the index clear), so the
// order of each state's outputs and the rounding of its sums are fixed by that
// state alone: a result is the same whatever else shares the tick.
//
// Order of a tick: fused runs; branching gates (index clear, index build,
// count, scan, write); measurements (reduce, decide, write).  Items of
// different states never touch each other's memory, so the families need no
// ordering among themselves.
#include "batch_units.h"
#include "bitslice_tile.h"
#include "entry_ops.h"
#include "u2_lds.h"

namespace sparsesim {
namespace {

using ent::cadd;
using ent::hash_label;
using ent::survives;


using ent::ctrl_ok;

__device__ __forceinline__ uint32_t find_label2(const BItem& it, uint64_t lo, uint64_t hi) {
  const uint64_t h = hash_label(lo, hi);
  const uint32_t fp = (uint32_t)(h >> 32);
  uint64_t slot = h & it.mask;
  for (uint64_t p = 0; p <= it.mask; ++p) {
    const uint64_t s = it.table[slot];
    if (s == kEmptySlot) return kNoPartner;
    if ((uint32_t)(s >> 32) == fp) {
      const uint32_t j = (uint32_t)s;
      if (it.in.key_lo[j] == lo && (!it.wide || it.in.key_hi[j] == hi)) return j;
    }
    slot = (slot + 1) & it.mask;
  }
  return kNoPartner;
}

using ent::pivot_set;

// Eq. 2 for one entry, given its partner (label ^ x): mode 0 passes through, 1
// emits the pair (o0 for the pivot-0 label b0, o1 for b0 ^ x), 2 emits nothing.
__device__ __forceinline__ int u2_entry(const BItem& it, uint64_t lo, uint64_t hi, double2 a, uint32_t j,
                                        double2* o0, double2* o1) {
  const ent::U2Out r = ent::u2_eval(it.u2, it.wide, it.in.amp, lo, hi, a, j);
  *o0 = r.o0;
  *o1 = r.o1;
  return r.mode;
}

template <typename T>
__device__ __forceinline__ T bsum(T v, T* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (unsigned s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return cadd(a, b); }

__device__ __forceinline__ uint32_t prefix012(uint32_t e, uint32_t* s_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t b1 = __ballot(e >= 1), b2 = __ballot(e >= 2);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const uint32_t pre = __popcll(b1 & lt) + __popcll(b2 & lt);
  if (lane == 0) s_wave[wid] = __popcll(b1) + __popcll(b2);
  __syncthreads();
  uint32_t woff = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t x = s_wave[w];
    woff += w < wid ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return woff + pre;
}

// ---- fused runs: one 2048-entry tile per unit, one wave per block ----------
// Bit-sliced runs take the register-plane tile (its planes in v100 and up,
// which the compiler may not allocate: amdgpu_num_vgpr counts pairs on
// gfx950, 40 = v0..v79; the clobber makes the kernel's VGPR count cover
// 131 planes).

// Fused runs: one unit (kChunk entries of one state) per block iteration, on
// the LDS-plane bit-sliced tile, or per entry for runs that form cannot take.
// (The register-plane tile of the single-state engine is not used here: its
// GPR-indexed plane accesses gave results that depended on which other
// states' tiles shared a SIMD, while the LDS-plane tile reproduces the
// single-state results in any mix.)
__global__ __launch_bounds__(64, 2) void kb_mono(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                              const uint32_t* __restrict__ units) {
  extern __shared__ uint32_t lds_all[];
  uint32_t* L = lds_all + threadIdx.x;
  const int n = (int)hdr->n_mono;
  if (n == 0) return;
  const uint32_t* u0 = units + hdr->mono_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = items[i];
    const uint64_t base = (uint64_t)(u - u0[i]) * kChunk;
    const uint32_t lim = (uint32_t)(it.nnz - base < kChunk ? it.nnz - base : kChunk);
    if (it.gops) {
      if (it.run.has_turns)
        bs::bs_tile<true>(it.in, base, lim, it.gops, it.ngroups, it.run, L);
      else
        bs::bs_tile<false>(it.in, base, lim, it.gops, it.ngroups, it.run, L);
      continue;
    }
    const bool phase = it.run_flags & kRunPhase, flip = it.run_flags & kRunFlip;
    for (uint32_t e = threadIdx.x; e < lim; e += 64) {
      const uint64_t idx = base + e;
      uint64_t lo = it.in.key_lo[idx], hi = it.wide ? it.in.key_hi[idx] : 0ull;
      double2 a = make_double2(0.0, 0.0);
      if (phase) a = it.in.amp[idx];
      for (uint32_t k = 0; k < it.n_dops; ++k) {
        const MonoDesc d = it.dops[k];
        const bool c = (lo & d.ctrl_lo) == d.ctrl_lo && (!it.wide || (hi & d.ctrl_hi) == d.ctrl_hi);
        const bool thi = it.wide && d.target >= 64;
        const uint64_t tbit = 1ull << (d.target & 63);
        const uint64_t w = thi ? hi : lo;
        if (d.flags & kHasPhase) {
          const double2 r = ent::cmul(a, ent::sel2((w & tbit) != 0, d.m1, d.m0));
          a = ent::sel2(c, r, a);
        }
        if (d.flags & kFlip) {
          const uint64_t f = c ? tbit : 0ull;
          if (thi) hi ^= f;
          else lo ^= f;
        }
      }
      if (flip) {
        it.in.key_lo[idx] = lo;
        if (it.wide) it.in.key_hi[idx] = hi;
      }
      if (phase) it.in.amp[idx] = a;
    }
  }
}

// ---- branching gates ---------------------------------------------------------
__global__ __launch_bounds__(256) void kb_fill(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                               const uint32_t* __restrict__ units) {
  const int n = (int)hdr->n_u2;
  if (n == 0) return;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->fill_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = u2[i];
    const uint64_t s0 = (uint64_t)(u - u0[i]) * kFillUnit;
    const uint64_t s1 = s0 + kFillUnit < it.mask + 1 ? s0 + kFillUnit : it.mask + 1;
    for (uint64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) it.table[s] = kEmptySlot;
  }
}

__global__ __launch_bounds__(256) void kb_build(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                const uint32_t* __restrict__ units) {
  const int n = (int)hdr->n_u2;
  if (n == 0) return;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->build_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = u2[i];
    const uint64_t e0 = (uint64_t)(u - u0[i]) * kChunk;
    const uint64_t e1 = e0 + kChunk < it.nnz ? e0 + kChunk : it.nnz;
    auto* table = reinterpret_cast<unsigned long long*>(it.table);
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      // Only entries under the controls with the pivot bit clear are indexed
      // (the partner look-ups come from the pivot-1 entries); every partner
      // slot starts empty.
      it.partner[e] = kNoPartner;
      const uint64_t lo = it.in.key_lo[e], hi = it.wide ? it.in.key_hi[e] : 0ull;
      if (!ctrl_ok(it.u2, lo, hi, it.wide) || pivot_set(it.u2, lo, hi, it.wide)) continue;
      const uint64_t h = hash_label(lo, hi);
      const unsigned long long val = ((h >> 32) << 32) | e;
      uint64_t slot = h & it.mask;
      for (uint64_t p = 0; p <= it.mask; ++p) {
        if (atomicCAS(&table[slot], (unsigned long long)kEmptySlot, val) == kEmptySlot) break;
        slot = (slot + 1) & it.mask;
      }
    }
  }
}

// Each entry under the controls with the pivot bit set looks up label ^ x;
// a hit records the two entries as each other's partner.
__global__ __launch_bounds__(256) void kb_u2_probe(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                   const uint32_t* __restrict__ units) {
  const int n = (int)hdr->n_u2;
  if (n == 0) return;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->build_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = u2[i];
    const uint64_t e0 = (uint64_t)(u - u0[i]) * kChunk;
    const uint64_t e1 = e0 + kChunk < it.nnz ? e0 + kChunk : it.nnz;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const uint64_t lo = it.in.key_lo[e], hi = it.wide ? it.in.key_hi[e] : 0ull;
      if (!ctrl_ok(it.u2, lo, hi, it.wide) || !pivot_set(it.u2, lo, hi, it.wide)) continue;
      const uint32_t j = find_label2(it, lo ^ it.u2.x_lo, it.wide ? (hi ^ it.u2.x_hi) : 0ull);
      if (j == kNoPartner) continue;
      it.partner[e] = j;
      it.partner[j] = (uint32_t)e;
    }
  }
}

__global__ __launch_bounds__(256) void kb_u2_count(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                   const uint32_t* __restrict__ units) {
  __shared__ uint32_t sh[256];
  const int n = (int)hdr->n_u2;
  if (n == 0) return;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->chunk_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = u2[i];
    const uint32_t c = u - u0[i];
    const uint64_t e0 = (uint64_t)c * kChunk;
    const uint64_t e1 = e0 + kChunk < it.nnz ? e0 + kChunk : it.nnz;
    uint32_t emit = 0;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const uint64_t lo = it.in.key_lo[e], hi = it.wide ? it.in.key_hi[e] : 0ull;
      double2 o0, o1;
      const int mode = u2_entry(it, lo, hi, it.in.amp[e], it.partner[e], &o0, &o1);
      if (mode == 0) emit += survives(o0, it.u2.eps) ? 1u : 0u;
      else if (mode == 1) emit += (survives(o0, it.u2.eps) ? 1u : 0u) + (survives(o1, it.u2.eps) ? 1u : 0u);
    }
    emit = bsum(emit, sh);
    if (threadIdx.x == 0) it.tot[c] = emit;
  }
}

// One block per item: exclusive scan of its unit counts; total -> tot[units]
// and, if it fits the capacity, the new entry count (else the overflow flag).
__global__ __launch_bounds__(256) void kb_u2_scan(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                  const uint32_t* __restrict__ units) {
  __shared__ uint32_t sh[256];
  const int n = (int)hdr->n_u2;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->chunk_u0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem& it = u2[i];
    const uint32_t nc = u0[i + 1] - u0[i];
    const uint32_t per = (nc + blockDim.x - 1) / blockDim.x;
    const uint32_t first = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t k = 0; k < per; ++k)
      if (first + k < nc) s += it.tot[first + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (unsigned off = 1; off < blockDim.x; off <<= 1) {
      const uint32_t x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
      __syncthreads();
      sh[threadIdx.x] += x;
      __syncthreads();
    }
    uint32_t run = sh[threadIdx.x] - s;
    for (uint32_t k = 0; k < per; ++k) {
      if (first + k < nc) {
        const uint32_t x = it.tot[first + k];
        it.tot[first + k] = run;
        run += x;
      }
    }
    if (threadIdx.x == blockDim.x - 1) {
      const uint32_t total = sh[threadIdx.x];
      it.tot[nc] = total;
      if (total > it.cap) it.ctl->status |= kStOverflow;
      else it.ctl->nnz[it.other] = total;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void kb_u2_write(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                   const uint32_t* __restrict__ units) {
  __shared__ uint32_t s_wave[4];
  const int n = (int)hdr->n_u2;
  if (n == 0) return;
  const BItem* u2 = items + hdr->n_mono;
  const uint32_t* u0 = units + hdr->chunk_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = u2[i];
    const uint32_t c = u - u0[i];
    if (it.tot[u0[i + 1] - u0[i]] > it.cap) continue;          // overflow: leave the state alone
    const uint64_t e0 = (uint64_t)c * kChunk;
    const uint64_t e1 = e0 + kChunk < it.nnz ? e0 + kChunk : it.nnz;
    uint64_t base = it.tot[c];
    for (uint64_t tile = e0; tile < e1; tile += blockDim.x) {
      const uint64_t e = tile + threadIdx.x;
      uint32_t cnt = 0;
      bool k0 = false, k1 = false;
      int mode = 2;
      uint64_t lo = 0, hi = 0;
      double2 o0 = make_double2(0.0, 0.0), o1 = o0;
      if (e < e1) {
        lo = it.in.key_lo[e];
        hi = it.wide ? it.in.key_hi[e] : 0ull;
        mode = u2_entry(it, lo, hi, it.in.amp[e], it.partner[e], &o0, &o1);
        if (mode == 0) k0 = survives(o0, it.u2.eps);
        if (mode == 1) {
          k0 = survives(o0, it.u2.eps);
          k1 = survives(o1, it.u2.eps);
        }
        cnt = (k0 ? 1u : 0u) + (k1 ? 1u : 0u);
      }
      uint32_t tile_total;
      uint64_t pos = base + prefix012(cnt, s_wave, &tile_total);
      if (mode == 0 && k0) {
        it.out.key_lo[pos] = lo;
        if (it.wide) it.out.key_hi[pos] = hi;
        it.out.amp[pos] = o0;
      } else if (mode == 1) {
        const bool v = pivot_set(it.u2, lo, hi, it.wide);
        const uint64_t lo0 = v ? lo ^ it.u2.x_lo : lo, hi0 = v ? hi ^ it.u2.x_hi : hi;
        if (k0) {
          it.out.key_lo[pos] = lo0;
          if (it.wide) it.out.key_hi[pos] = hi0;
          it.out.amp[pos] = o0;
          ++pos;
        }
        if (k1) {
          it.out.key_lo[pos] = lo0 ^ it.u2.x_lo;
          if (it.wide) it.out.key_hi[pos] = hi0 ^ it.u2.x_hi;
          it.out.amp[pos] = o1;
        }
      }
      base += tile_total;
    }
  }
}

// Branching gates of small states (at most kLdsU2Max entries), one item per
// block, partner index in LDS (lds::u2_block): the outputs and their order are
// those of the fill/build/probe/count/scan/write kernels above; more outputs
// than the capacity set the overflow flag (the state's current buffer is not
// written).
__global__ __launch_bounds__(1024) void kb_u2_lds(const BTick* __restrict__ hdr, const BItem* __restrict__ items) {
  __shared__ lds::Smem sm;
  const int n = (int)hdr->n_u2s;
  const BItem* u2s = items + hdr->n_mono + hdr->n_u2 + hdr->n_meas;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem& it = u2s[i];
    if (it.nnz > kLdsU2Max) {   // the host sends only small states here
      if (threadIdx.x == 0) it.ctl->status |= kStOverflow;
      continue;
    }
    const lds::Totals t = it.wide ? lds::u2_block<true>(it.in, it.out, (uint32_t)it.nnz, it.u2, it.cap, sm)
                                  : lds::u2_block<false>(it.in, it.out, (uint32_t)it.nnz, it.u2, it.cap, sm);
    if (threadIdx.x == 0) {
      if (t.out > it.cap) it.ctl->status |= kStOverflow;
      else it.ctl->nnz[it.other] = t.out;
    }
    __syncthreads();   // the next item reuses the LDS
  }
}

// ---- measurements ------------------------------------------------------------
// Entries of a measurement item's input.  The first measurement of a tick
// knows its count; a later step of a chain takes the count the previous step
// wrote (at most it.nnz, the count before the chain, from which its units
// were laid out: units past the count are empty and add nothing).
__device__ __forceinline__ uint64_t meas_nnz(const BItem& it) {
  if (it.chain == 0) return it.nnz;
  const uint64_t d = it.ctl->nnz[it.other ^ 1u];
  return d < it.nnz ? d : it.nnz;
}

__global__ __launch_bounds__(256) void kb_m_reduce(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                   const uint32_t* __restrict__ units) {
  __shared__ double2 shd[256];
  __shared__ uint32_t shu[256];
  const int n = (int)hdr->n_meas;
  if (n == 0) return;
  const BItem* m = items + hdr->n_mono + hdr->n_u2;
  const uint32_t* u0 = units + hdr->meas_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = m[i];
    const uint64_t nnz = meas_nnz(it);
    const uint32_t c = u - u0[i];
    const uint64_t e0 = (uint64_t)c * kChunk;
    const uint64_t e1 = e0 + kChunk < nnz ? e0 + kChunk : nnz;
    const bool qhi = it.wide && it.q >= 64;
    double p0 = 0.0, p1 = 0.0;
    uint32_t c1 = 0;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const uint64_t w = qhi ? it.in.key_hi[e] : it.in.key_lo[e];
      const double2 a = it.in.amp[e];
      const double p = a.x * a.x + a.y * a.y;
      if ((w >> (it.q & 63)) & 1ull) {
        p1 += p;
        ++c1;
      } else {
        p0 += p;
      }
    }
    const double2 s = bsum(make_double2(p0, p1), shd);
    const uint32_t cc = bsum(c1, shu);
    if (threadIdx.x == 0) {
      it.part[c] = s;
      it.cnt1[c] = cc;
    }
  }
}

__global__ __launch_bounds__(256) void kb_m_decide(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                   const uint32_t* __restrict__ units) {
  __shared__ double2 shd[256];
  __shared__ uint32_t shu[256];
  __shared__ int s_o;
  const int n = (int)hdr->n_meas;
  const BItem* m = items + hdr->n_mono + hdr->n_u2;
  const uint32_t* u0 = units + hdr->meas_u0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem& it = m[i];
    const uint64_t nnz = meas_nnz(it);
    const uint32_t nc = u0[i + 1] - u0[i];
    double2 acc = make_double2(0.0, 0.0);
    for (uint32_t k = threadIdx.x; k < nc; k += blockDim.x) acc = cadd(acc, it.part[k]);
    const double2 P = bsum(acc, shd);
    if (threadIdx.x == 0) {
      const double tot = P.x + P.y;
      int o = it.forced >= 0 ? it.forced : (it.u < P.x / tot ? 0 : 1);
      const double po = o ? P.y : P.x;
      double scale = 1.0 / sqrt(po);
      if (!(tot > 0.0) || !(po > 0.0)) {
        it.ctl->status |= kStMeasure;
        o = -1;
        scale = 0.0;
      }
      it.ctl->rec.p0 = P.x;
      it.ctl->rec.p1 = P.y;
      it.ctl->rec.scale = scale;
      it.ctl->rec.outcome = o;
      it.ctl->outcome = o;
      if (it.chain < kMaxChain) it.ctl->chain_out[it.chain] = o;
      s_o = o;
    }
    __syncthreads();
    const int o = s_o;
    const uint32_t per = (nc + blockDim.x - 1) / blockDim.x;
    const uint32_t first = threadIdx.x * per;
    auto count = [&](uint32_t k) -> uint32_t {
      const uint64_t b0 = (uint64_t)k * kChunk;
      const uint64_t b1 = b0 + kChunk < nnz ? b0 + kChunk : nnz;
      const uint32_t len = b0 < b1 ? (uint32_t)(b1 - b0) : 0u;
      return o == 1 ? it.cnt1[k] : (o == 0 ? len - it.cnt1[k] : 0u);
    };
    uint32_t s = 0;
    for (uint32_t k = 0; k < per; ++k)
      if (first + k < nc) s += count(first + k);
    shu[threadIdx.x] = s;
    __syncthreads();
    for (unsigned d = 1; d < blockDim.x; d <<= 1) {
      const uint32_t x = threadIdx.x >= d ? shu[threadIdx.x - d] : 0u;
      __syncthreads();
      shu[threadIdx.x] += x;
      __syncthreads();
    }
    uint32_t run = shu[threadIdx.x] - s;
    for (uint32_t k = 0; k < per; ++k) {
      if (first + k < nc) {
        it.tot[first + k] = run;
        run += count(first + k);
      }
    }
    if (threadIdx.x == blockDim.x - 1) it.ctl->nnz[it.other] = shu[threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void kb_m_write(const BTick* __restrict__ hdr, const BItem* __restrict__ items,
                                                  const uint32_t* __restrict__ units) {
  __shared__ uint32_t s_wave[4];
  const int n = (int)hdr->n_meas;
  if (n == 0) return;
  const BItem* m = items + hdr->n_mono + hdr->n_u2;
  const uint32_t* u0 = units + hdr->meas_u0;
  const uint32_t total = u0[n];
  for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int i = find_item(u0, n, u);
    const BItem& it = m[i];
    const int o = it.ctl->rec.outcome;
    if (o < 0) continue;
    const double scale = it.ctl->rec.scale;
    const uint64_t nnz = meas_nnz(it);
    const uint32_t c = u - u0[i];
    const uint64_t e0 = (uint64_t)c * kChunk;
    const uint64_t e1 = e0 + kChunk < nnz ? e0 + kChunk : nnz;
    const bool qhi = it.wide && it.q >= 64;
    uint64_t base = it.tot[c];
    for (uint64_t tile = e0; tile < e1; tile += blockDim.x) {
      const uint64_t e = tile + threadIdx.x;
      bool keep = false;
      uint64_t lo = 0, hi = 0;
      if (e < e1) {
        lo = it.in.key_lo[e];
        hi = it.wide ? it.in.key_hi[e] : 0ull;
        keep = (int)(((qhi ? hi : lo) >> (it.q & 63)) & 1ull) == o;
      }
      uint32_t tile_total;
      const uint64_t pos = base + prefix012(keep ? 1u : 0u, s_wave, &tile_total);
      if (keep) {
        const double2 a = it.in.amp[e];
        it.out.key_lo[pos] = lo;
        if (it.wide) it.out.key_hi[pos] = hi;
        it.out.amp[pos] = make_double2(a.x * scale, a.y * scale);
      }
      base += tile_total;
    }
  }
}

}  // namespace

// A tick's kernels, in order, on fixed grids (capturable); families with no
// items this tick can be left out.
void launch_batch_tick(hipStream_t st, const BTick* hdr, const BItem* items, const uint32_t* units, int grid,
                       uint32_t families) {
  const size_t lds = (size_t)kMaxPlanes * 64 * 4;
  if (families & kFamMono) hipLaunchKernelGGL(kb_mono, dim3(grid), dim3(64), lds, st, hdr, items, units);
  if (families & kFamU2) {
    hipLaunchKernelGGL(kb_fill, dim3(grid), dim3(256), 0, st, hdr, items, units);
    hipLaunchKernelGGL(kb_build, dim3(grid), dim3(256), 0, st, hdr, items, units);
    hipLaunchKernelGGL(kb_u2_probe, dim3(grid), dim3(256), 0, st, hdr, items, units);
    hipLaunchKernelGGL(kb_u2_count, dim3(grid), dim3(256), 0, st, hdr, items, units);
    hipLaunchKernelGGL(kb_u2_scan, dim3(grid), dim3(256), 0, st, hdr, items, units);
    hipLaunchKernelGGL(kb_u2_write, dim3(grid), dim3(256), 0, st, hdr, items, units);
  }
  if (families & kFamU2s)
    hipLaunchKernelGGL(kb_u2_lds, dim3(grid < 256 ? grid : 256), dim3(lds::kThreads), 0, st, hdr, items);
  if (families & kFamMeas) launch_batch_meas(st, hdr, items, units, grid);
}

void launch_batch_meas(hipStream_t st, const BTick* hdr, const BItem* items, const uint32_t* units, int grid) {
  hipLaunchKernelGGL(kb_m_reduce, dim3(grid), dim3(256), 0, st, hdr, items, units);
  hipLaunchKernelGGL(kb_m_decide, dim3(grid), dim3(256), 0, st, hdr, items, units);
  hipLaunchKernelGGL(kb_m_write, dim3(grid), dim3(256), 0, st, hdr, items, units);
}

}  // namespace sparsesim
