// HIP kernels of libsparsesim for gfx950 (wave64).
//
// The state is a structure-of-arrays list of (label, amplitude) pairs.  Every
// kernel reads the live entry count from device memory, so the host never has
// to know it to launch work.  Kernels that change the entry count (branching
// gates, measurement) are "chunked": block b owns the contiguous entry range
// [b*chunk, (b+1)*chunk) with chunk fixed per kernel (chunk_len), counts what it
// will emit, a one-block scan turns the counts into output offsets, and the
// write kernel emits in entry order.  Output order is therefore a fixed
// function of the input order: runs are deterministic and no floating-point
// value is ever accumulated with atomics.
//
// Arithmetic is fixed so that results match a plain sequential evaluation:
// complex products are (a.re*b.re - a.im*b.im, a.re*b.im + a.im*b.re), sums of
// two products are evaluated left to right, |a|^2 = re*re + im*im, and the
// library is compiled with -ffp-contract=off.
#include "entry_ops.h"
#include "u2_lds.h"

namespace sparsesim {
namespace {

using ent::cadd;
using ent::cmul;
using ent::hash_label;
using ent::sel2;
using ent::survives;

// Entries per block of a chunked launch of nb blocks: `per`, or an even split
// when nb blocks of `per` do not cover n.  The host sizes the grid from its
// bound on n (at least n), so block ranges, and every sum grouped by block,
// depend on n alone and not on where the host last read the count.
__device__ __forceinline__ uint64_t chunk_len(uint64_t n, uint64_t nb, uint64_t per) {
  const uint64_t even = (n + nb - 1) / nb;
  return even > per ? even : per;
}

__device__ __forceinline__ void chunk_range(uint64_t n, uint64_t per, uint64_t& begin, uint64_t& end) {
  const uint64_t chunk = chunk_len(n, gridDim.x, per);
  begin = (uint64_t)blockIdx.x * chunk;
  end = begin + chunk < n ? begin + chunk : n;
  if (begin > end) begin = end;
}

// Exclusive prefix over the block of per-thread counts e in {0,1,2}, in
// thread order.  Returns the thread's offset; *total gets the block sum.
// Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_prefix012(uint32_t e, uint32_t* s_wave, uint32_t* total) {
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

// Sum over the block in a fixed order (deterministic): a butterfly within
// each wave, then the waves' sums in wave order.  sh needs one slot per wave.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_xor(v.x, o), y = __shfl_xor(v.y, o);
    v = make_double2(v.x + x, v.y + y);
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  const int nw = blockDim.x >> 6;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  for (int w = 1; w < nw; ++w) r = r + sh[w];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double2 operator+(double2 a, double2 b) { return cadd(a, b); }

// ---------------------------------------------------------------------------
__global__ void k_set_basis(Buf b, uint64_t* nnz, uint64_t lo, uint64_t hi) {
  b.key_lo[0] = lo;
  if (b.key_hi) b.key_hi[0] = hi;
  b.amp[0] = make_double2(1.0, 0.0);
  *nnz = 1;
}

__global__ void k_fill(uint64_t* __restrict__ p, uint64_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Fused phase/permutation pass (Sec. 3.2): each label takes every gate of the
// run in order, G_n o ... o G_1, entirely in registers; one read and one
// write of the entry per run.  Gate descriptors are wave-uniform.
template <bool WIDE, int ITEMS>
__global__ __launch_bounds__(256) void k_mono(Buf b, const uint64_t* __restrict__ nnz_p,
                                              const MonoDesc* __restrict__ g, uint32_t ng, uint32_t rf,
                                              uint32_t bpe, Ctl* ctl) {
  const uint64_t n = *nnz_p;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd((unsigned long long*)&ctl->updates, (unsigned long long)(n * ng));
    atomicAdd((unsigned long long*)&ctl->mono_bytes, (unsigned long long)(n * bpe));
    atomicAdd((unsigned long long*)&ctl->mono_updates, (unsigned long long)(n * ng));
  }
  const bool run_phase = rf & kRunPhase, run_flip = rf & kRunFlip;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * ITEMS;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x * ITEMS; base < n; base += stride) {
    uint64_t lo[ITEMS], hi[ITEMS];
    double2 a[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint64_t idx = base + (uint64_t)i * blockDim.x + threadIdx.x;
      const bool ok = idx < n;
      lo[i] = ok ? b.key_lo[idx] : 0ull;
      hi[i] = (WIDE && ok) ? b.key_hi[idx] : 0ull;
      a[i] = make_double2(0.0, 0.0);
      if (ok && run_phase) a[i] = b.amp[idx];
    }
    for (uint32_t j = 0; j < ng; ++j) {
      const MonoDesc d = g[j];
      const uint32_t t = d.target;
      const bool thi = WIDE && t >= 64;
      const uint64_t tbit = 1ull << (t & 63);
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        bool c = (lo[i] & d.ctrl_lo) == d.ctrl_lo;
        if (WIDE) c = c && ((hi[i] & d.ctrl_hi) == d.ctrl_hi);
        const uint64_t w = thi ? hi[i] : lo[i];
        if (d.flags & kHasPhase) {
          const double2 m = sel2((w & tbit) != 0, d.m1, d.m0);
          const double2 r = cmul(a[i], m);
          a[i] = sel2(c, r, a[i]);
        }
        if (d.flags & kFlip) {
          const uint64_t f = c ? tbit : 0ull;
          if (thi)
            hi[i] ^= f;
          else
            lo[i] ^= f;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const uint64_t idx = base + (uint64_t)i * blockDim.x + threadIdx.x;
      if (idx < n) {
        if (run_flip) {
          b.key_lo[idx] = lo[i];
          if (WIDE) b.key_hi[idx] = hi[i];
        }
        if (run_phase) b.amp[idx] = a[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Hash index: open addressing with linear probing over a power-of-two table
// of 64-bit slots (fingerprint << 32 | entry index), claimed with 64-bit CAS.
// Labels are unique, so an insert never meets its own label.
//
// Only the entries a partner look-up can ask for are indexed: those under
// the op's controls with the pivot bit clear (the look-ups come from their
// partners, whose pivot bit is set).  Every entry's partner slot starts empty.
// Block sums of two per-thread counters added to dst[0], dst[1] by thread 0
// (one atomic pair per block); nothing when dst is null (counting off).
__device__ __forceinline__ void add_counters(unsigned long long* dst, uint32_t a, uint32_t b) {
  __shared__ uint32_t sh_a[4], sh_b[4];
  if (!dst) return;   // uniform: a kernel argument
  const uint32_t x = block_sum(a, sh_a), y = block_sum(b, sh_b);
  if (threadIdx.x == 0) {
    if (x) atomicAdd(dst, (unsigned long long)x);
    if (y) atomicAdd(dst + 1, (unsigned long long)y);
  }
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_index_build(Buf b, const uint64_t* __restrict__ nnz_p,
                                                     unsigned long long* table, uint64_t mask, U2Desc d,
                                                     uint32_t* __restrict__ partner, unsigned long long* count) {
  const uint64_t n = *nnz_p;
  uint32_t inserts = 0, cas = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    partner[i] = kNoPartner;
    const uint64_t lo = b.key_lo[i];
    const uint64_t hi = WIDE ? b.key_hi[i] : 0ull;
    bool c = (lo & d.ctrl_lo) == d.ctrl_lo;
    if (WIDE) c = c && ((hi & d.ctrl_hi) == d.ctrl_hi);
    const uint64_t w = (WIDE && d.target >= 64) ? hi : lo;
    if (!c || ((w >> (d.target & 63)) & 1ull)) continue;
    const uint64_t h = hash_label(lo, hi);
    const unsigned long long val = ((h >> 32) << 32) | i;
    uint64_t slot = h & mask;
    ++inserts;
    for (uint64_t p = 0; p <= mask; ++p) {
      ++cas;
      if (atomicCAS(&table[slot], (unsigned long long)kEmptySlot, val) == kEmptySlot) break;
      slot = (slot + 1) & mask;
    }
  }
  add_counters(count, inserts, cas);
}

template <bool WIDE>
__device__ __forceinline__ uint32_t find_label(const Buf& b, const uint64_t* __restrict__ table, uint64_t mask,
                                               uint64_t lo, uint64_t hi, uint32_t& steps) {
  const uint64_t h = hash_label(lo, hi);
  const uint32_t fp = (uint32_t)(h >> 32);
  uint64_t slot = h & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    const uint64_t s = table[slot];
    ++steps;
    if (s == kEmptySlot) return kNoPartner;
    if ((uint32_t)(s >> 32) == fp) {
      const uint32_t j = (uint32_t)s;
      if (b.key_lo[j] == lo && (!WIDE || b.key_hi[j] == hi)) return j;
    }
    slot = (slot + 1) & mask;
  }
  return kNoPartner;
}

// Partner look-up (Sec. 3.1: at most one per label): each entry under the
// controls with the pivot bit set looks up label ^ x among the indexed
// entries; when found, both entries record each other (a pivot-0 entry has at
// most one such partner, so the writes never collide).
template <bool WIDE>
__global__ __launch_bounds__(256) void k_u2_probe(Buf b, const uint64_t* __restrict__ nnz_p,
                                                  const uint64_t* __restrict__ table, uint64_t mask, U2Desc d,
                                                  uint32_t* __restrict__ partner, unsigned long long* count) {
  const uint64_t n = *nnz_p;
  uint32_t lookups = 0, steps = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t lo = b.key_lo[i];
    const uint64_t hi = WIDE ? b.key_hi[i] : 0ull;
    bool c = (lo & d.ctrl_lo) == d.ctrl_lo;
    if (WIDE) c = c && ((hi & d.ctrl_hi) == d.ctrl_hi);
    const uint64_t w = (WIDE && d.target >= 64) ? hi : lo;
    if (!c || !((w >> (d.target & 63)) & 1ull)) continue;
    ++lookups;
    const uint32_t j = find_label<WIDE>(b, table, mask, lo ^ d.x_lo, WIDE ? (hi ^ d.x_hi) : 0ull, steps);
    if (j == kNoPartner) continue;
    partner[i] = j;
    partner[j] = (uint32_t)i;
  }
  add_counters(count, lookups, steps);
}

// The count, write and single-pass kernels take partner == null for a gate
// whose partner mask touches a qubit that is the same in every entry: then no
// entry has a partner, and no index is built or probed.
template <bool WIDE>
__device__ __forceinline__ bool pivot_set(const U2Desc& d, uint64_t lo, uint64_t hi) {
  return ent::pivot_set(d, lo, hi, WIDE);
}

using ent::U2Out;
template <bool WIDE>
__device__ __forceinline__ U2Out u2_eval(const Buf& b, const U2Desc& d, uint64_t lo, uint64_t hi, double2 a,
                                         uint32_t j) {
  return ent::u2_eval(d, WIDE, b.amp, lo, hi, a, j);
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_u2_count(Buf b, const uint64_t* __restrict__ nnz_p, U2Desc d,
                                                  const uint32_t* __restrict__ partner, uint32_t* __restrict__ tot,
                                                  Ctl* ctl) {
  __shared__ uint32_t sh[256];
  __shared__ double2 shm[4];   // one slot per wave
  const uint64_t n = *nnz_p;
  uint64_t begin, end;
  chunk_range(n, kTwoPassChunk, begin, end);
  uint32_t emit = 0, dropped = 0;
  double mass = 0.0;
  for (uint64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
    const uint64_t lo = b.key_lo[i];
    const uint64_t hi = WIDE ? b.key_hi[i] : 0ull;
    const U2Out r = u2_eval<WIDE>(b, d, lo, hi, b.amp[i], partner ? partner[i] : kNoPartner);
    if (r.mode == 0) {
      const bool k = survives(r.o0, d.eps);
      emit += k ? 1u : 0u;
      dropped += k ? 0u : 1u;
      mass += ent::dropped_mass(r.o0, k);
    } else if (r.mode == 1) {
      const bool k0 = survives(r.o0, d.eps), k1 = survives(r.o1, d.eps);
      emit += (k0 ? 1u : 0u) + (k1 ? 1u : 0u);
      dropped += (k0 ? 0u : 1u) + (k1 ? 0u : 1u);
      mass += ent::dropped_mass(r.o0, k0) + ent::dropped_mass(r.o1, k1);
    }
  }
  emit = block_sum(emit, sh);
  dropped = block_sum(dropped, sh);
  mass = block_sum(make_double2(mass, 0.0), shm).x;
  if (threadIdx.x == 0) {
    tot[blockIdx.x] = emit;
    if (dropped) {
      atomicAdd((unsigned long long*)&ctl->st_pruned, (unsigned long long)dropped);
      atomicAdd(&ctl->st_mass, mass);
    }
    if (blockIdx.x == 0) {
      atomicAdd((unsigned long long*)&ctl->st_updates, (unsigned long long)n);
      atomicAdd((unsigned long long*)&ctl->pass_bytes[0], (unsigned long long)(n * (WIDE ? 32u : 24u)));
    }
  }
}

// One block: exclusive scan of per-block counts in place; the total becomes
// the entry count of the output buffer.  The count pass's staged counters
// are committed if the total fits cap (otherwise the gate is rejected and
// they are discarded).
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ tot, int nb, uint64_t* nnz_out, Ctl* ctl,
                                               uint32_t entry_bytes, uint64_t cap) {
  __shared__ uint32_t sh[1024];
  const int per = (nb + blockDim.x - 1) / blockDim.x;
  const int first = threadIdx.x * per;
  uint32_t s = 0;
  for (int k = 0; k < per; ++k)
    if (first + k < nb) s += tot[first + k];
  sh[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over thread sums.
  for (unsigned off = 1; off < blockDim.x; off <<= 1) {
    const uint32_t x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = sh[threadIdx.x] - s;
  for (int k = 0; k < per; ++k) {
    if (first + k < nb) {
      const uint32_t x = tot[first + k];
      tot[first + k] = run;
      run += x;
    }
  }
  if (threadIdx.x == blockDim.x - 1) {
    const uint64_t total = sh[threadIdx.x];
    *nnz_out = total;
    if (total <= cap) {
      if (total > ctl->peak) ctl->peak = total;
      ctl->pass_bytes[1] += total * entry_bytes;   // the write pass's output
      ctl->updates += ctl->st_updates;
      ctl->pruned += ctl->st_pruned;
      ctl->pruned_mass += ctl->st_mass;
    }
    ctl->st_updates = 0;
    ctl->st_pruned = 0;
    ctl->st_mass = 0.0;
  }
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_u2_write(Buf in, Buf out, const uint64_t* __restrict__ nnz_p,
                                                  const uint32_t* __restrict__ partner,
                                                  const uint32_t* __restrict__ off, U2Desc d, Ctl* ctl) {
  __shared__ uint32_t s_wave[16];
  const uint64_t n = *nnz_p;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd((unsigned long long*)&ctl->pass_bytes[1], (unsigned long long)(n * (WIDE ? 32u : 24u)));
  uint64_t begin, end;
  chunk_range(n, kTwoPassChunk, begin, end);
  uint64_t base = off[blockIdx.x];
  for (uint64_t tile = begin; tile < end; tile += blockDim.x) {
    const uint64_t i = tile + threadIdx.x;
    uint32_t e = 0;
    bool k0 = false, k1 = false;
    U2Out r;
    uint64_t lo = 0, hi = 0;
    r.mode = 2;
    if (i < end) {
      lo = in.key_lo[i];
      hi = WIDE ? in.key_hi[i] : 0ull;
      r = u2_eval<WIDE>(in, d, lo, hi, in.amp[i], partner ? partner[i] : kNoPartner);
      if (r.mode == 0) {
        k0 = survives(r.o0, d.eps);
      } else if (r.mode == 1) {
        k0 = survives(r.o0, d.eps);
        k1 = survives(r.o1, d.eps);
      }
      e = (k0 ? 1u : 0u) + (k1 ? 1u : 0u);
    }
    uint32_t tile_total;
    uint64_t pos = base + block_prefix012(e, s_wave, &tile_total);
    if (r.mode == 0) {
      if (k0) {
        out.key_lo[pos] = lo;
        if (WIDE) out.key_hi[pos] = hi;
        out.amp[pos] = r.o0;
      }
    } else if (r.mode == 1) {
      const bool v = pivot_set<WIDE>(d, lo, hi);
      const uint64_t lo0 = v ? lo ^ d.x_lo : lo, hi0 = v ? hi ^ d.x_hi : hi;
      if (k0) {
        out.key_lo[pos] = lo0;
        if (WIDE) out.key_hi[pos] = hi0;
        out.amp[pos] = r.o0;
        ++pos;
      }
      if (k1) {
        out.key_lo[pos] = lo0 ^ d.x_lo;
        if (WIDE) out.key_hi[pos] = hi0 ^ d.x_hi;
        out.amp[pos] = r.o1;
      }
    }
    base += tile_total;
  }
}

// Single-pass branching gate, for states whose outputs are known to fit:
// each block evaluates one tile of 256 ITEMS entries once (Eq. 2 with T_eps, the
// results held in registers) and finds where its outputs go by a chained scan
// over the tiles: it publishes its tile's output count, adds its
// predecessors' counts back to the first published inclusive prefix,
// publishes its own inclusive prefix, then writes.  Blocks take tile numbers
// from a counter in the order they start, so a tile waited on always belongs
// to a block already running; the wait is bounded even so (a block that gives
// up sets error bit 2 and its outputs are wrong, but the kernel ends).  A
// status word packs (epoch, flag, count) and is read and written atomically at
// device scope, so no fence is needed; the epoch tells this launch's words
// from those of earlier launches.  Output order is input order, as in the
// two-pass form.
constexpr uint64_t kStAgg = 1ull << 32, kStPrefix = 2ull << 32;
constexpr uint32_t kSpinMax = 1u << 22;

__device__ __forceinline__ uint64_t st_word(uint32_t epoch, uint64_t flag, uint32_t v) {
  return ((uint64_t)epoch << 34) | flag | v;
}

// Tiles of 512, 1024 or 2048 entries (ITEMS = 2, 4, 8): the larger tiles hold
// more registers (2048: two waves per SIMD), the smaller ones put more blocks
// in flight, which is what states of up to a few million entries need.
template <bool WIDE, int ITEMS>
__global__ __launch_bounds__(256) void k_u2_fused(Buf in, Buf out, const uint64_t* __restrict__ nnz_p,
                                                  const uint32_t* __restrict__ partner, U2Desc d, Ctl* ctl,
                                                  uint64_t* status, uint32_t ticket_base, uint32_t epoch,
                                                  uint64_t* nnz_out, uint64_t* __restrict__ table,
                                                  uint64_t clear_slots) {
  constexpr int kItems = ITEMS;
  constexpr uint32_t kTile = 256u * ITEMS;
  __shared__ uint32_t s_wave[16];
  __shared__ uint32_t sh[256];
  __shared__ double2 shm[4];   // one slot per wave
  __shared__ uint32_t s_tile, s_excl;
  const uint64_t n = *nnz_p;
  // This gate is done with the hash index: empty its first clear_slots slots
  // for the next branching gate (every block, by block index).
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < clear_slots;
       k += (uint64_t)gridDim.x * blockDim.x)
    table[k] = kEmptySlot;
  if (threadIdx.x == 0) s_tile = atomicAdd(&ctl->ticket, 1u) - ticket_base;
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= gridDim.x) {   // the counter and the host's base disagree: touch nothing
    if (threadIdx.x == 0) atomicOr(&ctl->error, 2u);
    return;
  }
  const uint64_t begin = (uint64_t)tile * kTile;
  U2Out r[kItems];
  uint64_t lo[kItems], hi[kItems];
  uint32_t pos[kItems];
  bool k0[kItems], k1[kItems];
  uint32_t run = 0, dropped = 0;
  double mass = 0.0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint64_t i = begin + (uint64_t)k * 256 + threadIdx.x;
    r[k].mode = 2;
    k0[k] = k1[k] = false;
    lo[k] = hi[k] = 0;
    if (i < n) {
      lo[k] = in.key_lo[i];
      hi[k] = WIDE ? in.key_hi[i] : 0ull;
      r[k] = u2_eval<WIDE>(in, d, lo[k], hi[k], in.amp[i], partner ? partner[i] : kNoPartner);
      if (r[k].mode == 0) {
        k0[k] = survives(r[k].o0, d.eps);
        dropped += k0[k] ? 0u : 1u;
        mass += ent::dropped_mass(r[k].o0, k0[k]);
      } else if (r[k].mode == 1) {
        k0[k] = survives(r[k].o0, d.eps);
        k1[k] = survives(r[k].o1, d.eps);
        dropped += (k0[k] ? 0u : 1u) + (k1[k] ? 0u : 1u);
        mass += ent::dropped_mass(r[k].o0, k0[k]) + ent::dropped_mass(r[k].o1, k1[k]);
      }
    }
    uint32_t tt;
    pos[k] = run + block_prefix012((k0[k] ? 1u : 0u) + (k1[k] ? 1u : 0u), s_wave, &tt);
    run += tt;
  }
  dropped = block_sum(dropped, sh);
  mass = block_sum(make_double2(mass, 0.0), shm).x;
  // Publish this tile's count, then the first wave looks back 64 tiles per
  // poll (lane l reads tile - 1 - l) and adds counts back to the nearest
  // published inclusive prefix; positions before tile 0 count as a prefix of 0.
  if (threadIdx.x == 0) {
    if (dropped) {
      atomicAdd((unsigned long long*)&ctl->pruned, (unsigned long long)dropped);
      atomicAdd(&ctl->pruned_mass, mass);
    }
    __hip_atomic_store(&status[tile], st_word(epoch, tile == 0 ? kStPrefix : kStAgg, run), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if (tile == 0) atomicAdd((unsigned long long*)&ctl->updates, (unsigned long long)n);
  }
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t excl = 0;
    int64_t hi_tile = (int64_t)tile - 1;
    uint32_t spins = 0;
    while (hi_tile >= 0) {
      const int64_t j = hi_tile - lane;
      const uint64_t v = j >= 0 ? __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : st_word(epoch, kStPrefix, 0);
      const bool ready = (uint32_t)(v >> 34) == epoch;
      const uint64_t pmask = __ballot(ready && (v & kStPrefix));
      const uint64_t nready = __ballot(!ready);
      const int first = pmask ? __builtin_ctzll(pmask) : 63;   // nearest prefix in the window, else all 64
      const uint64_t need = first == 63 ? ~0ull : ((2ull << first) - 1);
      if (nready & need) {
        if (++spins > kSpinMax) {
          if (lane == 0) atomicOr(&ctl->error, 2u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      uint32_t x = lane <= first ? (uint32_t)v : 0u;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
      excl += x;
      if (pmask) break;
      hi_tile -= 64;
    }
    if (lane == 0) {
      if (tile != 0)
        __hip_atomic_store(&status[tile], st_word(epoch, kStPrefix, excl + run), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      s_excl = excl;
      if (tile == gridDim.x - 1) {
        const uint32_t eb = WIDE ? 32u : 24u;
        const uint64_t total = (uint64_t)excl + run;
        *nnz_out = total;
        if (total > ctl->peak) ctl->peak = total;
        atomicAdd((unsigned long long*)&ctl->pass_bytes[1], (unsigned long long)((n + total) * eb));
      }
    }
  }
  __syncthreads();
  const uint64_t base = s_excl;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    uint64_t p = base + pos[k];
    if (r[k].mode == 0) {
      if (k0[k]) {
        out.key_lo[p] = lo[k];
        if (WIDE) out.key_hi[p] = hi[k];
        out.amp[p] = r[k].o0;
      }
    } else if (r[k].mode == 1) {
      const bool v = pivot_set<WIDE>(d, lo[k], hi[k]);
      const uint64_t lo0 = v ? lo[k] ^ d.x_lo : lo[k], hi0 = v ? hi[k] ^ d.x_hi : hi[k];
      if (k0[k]) {
        out.key_lo[p] = lo0;
        if (WIDE) out.key_hi[p] = hi0;
        out.amp[p] = r[k].o0;
        ++p;
      }
      if (k1[k]) {
        out.key_lo[p] = lo0 ^ d.x_lo;
        if (WIDE) out.key_hi[p] = hi0 ^ d.x_hi;
        out.amp[p] = r[k].o1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Branching gate on a state of at most kLdsU2Max entries in one block, its
// partner index in LDS (lds::u2_block): same outputs, order and counters as
// the index-build / probe / single-pass kernels, in one launch.
template <bool WIDE>
__global__ __launch_bounds__(1024) void k_u2_lds(Buf in, Buf out, const uint64_t* __restrict__ nnz_p, U2Desc d,
                                                 Ctl* ctl, uint64_t* nnz_out) {
  __shared__ lds::Smem sm;
  const uint64_t n = *nnz_p;
  if (n > kLdsU2Max) {   // the host launches this kernel only below the bound
    if (threadIdx.x == 0) atomicOr(&ctl->error, 4u);
    return;
  }
  // Outputs number at most 2 n, which the host has checked against the
  // capacity, so the bound passed here never refuses a write.
  const lds::Totals t = lds::u2_block<WIDE>(in, out, (uint32_t)n, d, ~0ull, sm);
  if (threadIdx.x == 0) {
    if (t.dropped) {
      atomicAdd((unsigned long long*)&ctl->pruned, (unsigned long long)t.dropped);
      atomicAdd(&ctl->pruned_mass, t.mass);
    }
    atomicAdd((unsigned long long*)&ctl->updates, (unsigned long long)n);
    for (int k = 0; k < 4; ++k)
      if (t.ix[k]) atomicAdd((unsigned long long*)&ctl->ix[k], (unsigned long long)t.ix[k]);
    *nnz_out = t.out;
    if (t.out > ctl->peak) ctl->peak = t.out;
    atomicAdd((unsigned long long*)&ctl->pass_bytes[4], (unsigned long long)((n + t.out) * (WIDE ? 32u : 24u)));
  }
}

// ---------------------------------------------------------------------------
// Measurement (Born rule): per-block sums of |a|^2 split by the measured bit,
// a one-block decision, then an ordered compaction that scales the survivors.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_measure_reduce(Buf b, const uint64_t* __restrict__ nnz_p, uint32_t q,
                                                        double2* __restrict__ part, uint32_t* __restrict__ cnt1) {
  __shared__ double2 shd[256];
  __shared__ uint32_t shu[256];
  const uint64_t n = *nnz_p;
  uint64_t begin, end;
  chunk_range(n, kMeasChunk, begin, end);
  double p0 = 0.0, p1 = 0.0;
  uint32_t c1 = 0;
  const bool qhi = WIDE && q >= 64;
  for (uint64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
    const uint64_t w = qhi ? b.key_hi[i] : b.key_lo[i];
    const double2 a = b.amp[i];
    const double p = a.x * a.x + a.y * a.y;
    if ((w >> (q & 63)) & 1ull) {
      p1 += p;
      ++c1;
    } else {
      p0 += p;
    }
  }
  const double2 s = block_sum(make_double2(p0, p1), shd);
  const uint32_t c = block_sum(c1, shu);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    cnt1[blockIdx.x] = c;
  }
}

__global__ __launch_bounds__(1024) void k_measure_decide(const double2* __restrict__ part,
                                                         const uint32_t* __restrict__ cnt1,
                                                         uint32_t* __restrict__ off, int nb,
                                                         const uint64_t* __restrict__ nnz_in, uint64_t* nnz_out,
                                                         double u, int32_t forced, MeasRec* rec, int32_t* outcome,
                                                         Ctl* ctl, uint32_t entry_bytes,
                                                         const uint32_t* __restrict__ in_off) {
  __shared__ double2 shd[1024];
  __shared__ uint32_t shu[1024];
  __shared__ int s_o;
  // Every load is issued before any sum needs it (a rolled loop would wait on
  // each in turn); the sums keep the per-thread order k, k + 1024, ...
  constexpr int kPer = kMaxBlocks / 1024;
  const uint64_t n = *nnz_in;
  double2 pv[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int k = threadIdx.x + 1024 * i;
    pv[i] = make_double2(0.0, 0.0);
    if (k < nb) pv[i] = part[k];
  }
  // Per-block kept counts need each block's input length: its uniform chunk,
  // or (in_off given) the range the previous measurement's write block
  // produced.  Thread t owns blocks [t per, (t + 1) per).
  const uint64_t chunk = chunk_len(n, nb, kMeasChunk);
  const int per = (nb + 1023) / 1024;
  const int first = threadIdx.x * per;
  uint32_t c1[kPer], len[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int bidx = first + i;
    c1[i] = len[i] = 0;
    if (i < per && bidx < nb) {
      c1[i] = cnt1[bidx];
      if (in_off) {
        len[i] = (uint32_t)((bidx + 1 < nb ? (uint64_t)in_off[bidx + 1] : n) - in_off[bidx]);
      } else {
        uint64_t bb = (uint64_t)bidx * chunk, be = bb + chunk < n ? bb + chunk : n;
        if (bb > be) bb = be;
        len[i] = (uint32_t)(be - bb);
      }
    }
  }
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < kPer; ++i) acc = cadd(acc, pv[i]);
  const double2 P = block_sum(acc, shd);
  if (threadIdx.x == 0) {
    const double tot = P.x + P.y;
    int o = forced >= 0 ? forced : (u < P.x / tot ? 0 : 1);
    const double po = o ? P.y : P.x;
    double scale = 1.0 / sqrt(po);
    if (!(tot > 0.0) || !(po > 0.0)) {
      atomicOr(&ctl->error, 1u);
      o = -1;
      scale = 0.0;
    }
    rec->p0 = P.x;
    rec->p1 = P.y;
    rec->scale = scale;
    rec->outcome = o;
    *outcome = o;
    s_o = o;
  }
  __syncthreads();
  const int o = s_o;
  // Output counts per block for the chosen outcome, then exclusive scan.
  uint32_t kept_b[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    kept_b[i] = o == 1 ? c1[i] : (o == 0 ? len[i] - c1[i] : 0u);
    s += kept_b[i];
  }
  // Inclusive scan of the per-thread counts: within each wave by shuffles,
  // then the preceding waves' totals.
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d);
    if (lane >= d) incl += y;
  }
  if (lane == 63) shu[wid] = incl;
  __syncthreads();
  uint32_t kept_total = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wid) incl += shu[w];
    kept_total += shu[w];
  }
  uint32_t run = incl - s;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int bidx = first + i;
    if (i < per && bidx < nb) {
      off[bidx] = run;
      run += kept_b[i];
    }
  }
  if (threadIdx.x == blockDim.x - 1) {
    const uint64_t kept = kept_total;
    *nnz_out = kept;
    // reduce: the label word holding the qubit and the amplitude of every
    // entry (none when the previous write formed the sums)
    if (!in_off) ctl->pass_bytes[2] += n * 24u;
    // write: that label word of every entry, the rest of each kept entry, and the kept entries written
    ctl->pass_bytes[3] += n * 8u + kept * (2u * entry_bytes - 8u);
  }
}

// Ordered compaction of the entries with the measured outcome, scaled.  The
// block's input range is its uniform chunk, or (in_off given) the range the
// previous measurement's write block produced.  With q_next >= 0 the block
// also forms the next measurement's sums over the entries it writes, in the
// same form as the reduce kernel (its output range is then that
// measurement's input range for this block).
template <bool WIDE>
__global__ __launch_bounds__(256) void k_measure_write(Buf in, Buf out, const uint64_t* __restrict__ nnz_p,
                                                       uint32_t q, const MeasRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ in_off, int32_t q_next,
                                                       double2* __restrict__ part_next,
                                                       uint32_t* __restrict__ cnt1_next) {
  __shared__ uint32_t s_wave[16];
  __shared__ double2 shd[256];
  __shared__ uint32_t shu[256];
  const uint64_t n = *nnz_p;
  uint64_t begin, end;
  if (in_off) {
    begin = in_off[blockIdx.x];
    end = blockIdx.x + 1 < gridDim.x ? in_off[blockIdx.x + 1] : n;
  } else {
    chunk_range(n, kMeasChunk, begin, end);
  }
  const int o = rec->outcome;
  const double scale = rec->scale;
  uint64_t base = off[blockIdx.x];
  const bool qhi = WIDE && q >= 64;
  const bool nhi = WIDE && q_next >= 64;
  double p0 = 0.0, p1 = 0.0;
  uint32_t c1 = 0;
  for (uint64_t tile = begin; tile < end; tile += blockDim.x) {
    const uint64_t i = tile + threadIdx.x;
    bool keep = false;
    uint64_t lo = 0, hi = 0;
    if (i < end && o >= 0) {
      lo = in.key_lo[i];
      hi = WIDE ? in.key_hi[i] : 0ull;
      const uint64_t w = qhi ? hi : lo;
      keep = (int)((w >> (q & 63)) & 1ull) == o;
    }
    uint32_t tile_total;
    const uint64_t pos = base + block_prefix012(keep ? 1u : 0u, s_wave, &tile_total);
    if (keep) {
      const double2 a = in.amp[i];
      const double2 v = make_double2(a.x * scale, a.y * scale);
      out.key_lo[pos] = lo;
      if (WIDE) out.key_hi[pos] = hi;
      out.amp[pos] = v;
      if (q_next >= 0) {
        const double p = v.x * v.x + v.y * v.y;
        if ((((nhi ? hi : lo) >> (q_next & 63)) & 1ull) != 0) {
          p1 += p;
          ++c1;
        } else {
          p0 += p;
        }
      }
    }
    base += tile_total;
  }
  if (q_next >= 0) {
    const double2 sum = block_sum(make_double2(p0, p1), shd);
    const uint32_t c = block_sum(c1, shu);
    if (threadIdx.x == 0) {
      part_next[blockIdx.x] = sum;
      cnt1_next[blockIdx.x] = c;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
void launch_set_basis(hipStream_t st, Buf b, uint64_t* nnz, uint64_t lo, uint64_t hi) {
  hipLaunchKernelGGL(k_set_basis, dim3(1), dim3(1), 0, st, b, nnz, lo, hi);
}

void launch_fill(hipStream_t st, uint64_t* p, uint64_t v, uint64_t n) {
  const uint64_t blocks = (n + 255) / 256;
  const int grid = (int)(blocks < 16384 ? (blocks ? blocks : 1) : 16384);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, p, v, n);
}

void launch_mono(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const MonoDesc* g, uint32_t ng,
                 uint32_t run_flags, uint32_t bytes_per_entry, Ctl* ctl, int grid, int block) {
  if (wide)
    hipLaunchKernelGGL((k_mono<true, 4>), dim3(grid), dim3(block), 0, st, b, nnz, g, ng, run_flags, bytes_per_entry,
                       ctl);
  else
    hipLaunchKernelGGL((k_mono<false, 4>), dim3(grid), dim3(block), 0, st, b, nnz, g, ng, run_flags, bytes_per_entry,
                       ctl);
}

void launch_index_build(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, uint64_t* table, uint64_t mask,
                        const U2Desc& d, uint32_t* partner, Ctl* ctl, int grid, int block) {
  auto* t = reinterpret_cast<unsigned long long*>(table);
  auto* count = ctl ? reinterpret_cast<unsigned long long*>(&ctl->ix[0]) : nullptr;
  if (wide)
    hipLaunchKernelGGL(k_index_build<true>, dim3(grid), dim3(block), 0, st, b, nnz, t, mask, d, partner, count);
  else
    hipLaunchKernelGGL(k_index_build<false>, dim3(grid), dim3(block), 0, st, b, nnz, t, mask, d, partner, count);
}

void launch_u2_probe(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const uint64_t* table, uint64_t mask,
                     const U2Desc& d, uint32_t* partner, Ctl* ctl, int grid, int block) {
  auto* count = ctl ? reinterpret_cast<unsigned long long*>(&ctl->ix[2]) : nullptr;
  if (wide)
    hipLaunchKernelGGL(k_u2_probe<true>, dim3(grid), dim3(block), 0, st, b, nnz, table, mask, d, partner, count);
  else
    hipLaunchKernelGGL(k_u2_probe<false>, dim3(grid), dim3(block), 0, st, b, nnz, table, mask, d, partner, count);
}

void launch_u2_count(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, const U2Desc& d, const uint32_t* partner,
                     uint32_t* tot, Ctl* ctl, int grid, int block) {
  if (wide)
    hipLaunchKernelGGL(k_u2_count<true>, dim3(grid), dim3(block), 0, st, b, nnz, d, partner, tot, ctl);
  else
    hipLaunchKernelGGL(k_u2_count<false>, dim3(grid), dim3(block), 0, st, b, nnz, d, partner, tot, ctl);
}

void launch_scan(hipStream_t st, uint32_t* tot, int nblocks, uint64_t* nnz_out, Ctl* ctl, uint32_t entry_bytes,
                 uint64_t cap) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, tot, nblocks, nnz_out, ctl, entry_bytes, cap);
}

void launch_u2_write(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const uint32_t* partner,
                     const uint32_t* off, const U2Desc& d, Ctl* ctl, int grid, int block) {
  if (wide)
    hipLaunchKernelGGL(k_u2_write<true>, dim3(grid), dim3(block), 0, st, in, out, nnz, partner, off, d, ctl);
  else
    hipLaunchKernelGGL(k_u2_write<false>, dim3(grid), dim3(block), 0, st, in, out, nnz, partner, off, d, ctl);
}

void launch_u2_fused(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const uint32_t* partner,
                     const U2Desc& d, Ctl* ctl, uint64_t* status, uint32_t ticket_base, uint32_t epoch,
                     uint64_t* nnz_out, uint64_t* table, uint64_t clear_slots, int grid, uint32_t tile) {
#define SPARSESIM_U2F(W, I)                                                                                    \
  hipLaunchKernelGGL((k_u2_fused<W, I>), dim3(grid), dim3(256), 0, st, in, out, nnz, partner, d, ctl, status, \
                     ticket_base, epoch, nnz_out, table, clear_slots)
  if (wide) {
    if (tile == 512) SPARSESIM_U2F(true, 2);
    else if (tile == 1024) SPARSESIM_U2F(true, 4);
    else SPARSESIM_U2F(true, 8);
  } else {
    if (tile == 512) SPARSESIM_U2F(false, 2);
    else if (tile == 1024) SPARSESIM_U2F(false, 4);
    else SPARSESIM_U2F(false, 8);
  }
#undef SPARSESIM_U2F
}

void launch_u2_lds(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, const U2Desc& d, Ctl* ctl,
                   uint64_t* nnz_out) {
  if (wide)
    hipLaunchKernelGGL(k_u2_lds<true>, dim3(1), dim3(lds::kThreads), 0, st, in, out, nnz, d, ctl, nnz_out);
  else
    hipLaunchKernelGGL(k_u2_lds<false>, dim3(1), dim3(lds::kThreads), 0, st, in, out, nnz, d, ctl, nnz_out);
}

void launch_measure_reduce(hipStream_t st, bool wide, Buf b, const uint64_t* nnz, uint32_t q, BlockScratch s,
                           int grid, int block) {
  if (wide)
    hipLaunchKernelGGL(k_measure_reduce<true>, dim3(grid), dim3(block), 0, st, b, nnz, q, s.part, s.cnt1);
  else
    hipLaunchKernelGGL(k_measure_reduce<false>, dim3(grid), dim3(block), 0, st, b, nnz, q, s.part, s.cnt1);
}

void launch_measure_decide(hipStream_t st, const double2* part, const uint32_t* cnt1, uint32_t* off, int nblocks,
                           const uint64_t* nnz_in, uint64_t* nnz_out, double u, int32_t forced, MeasRec* rec,
                           int32_t* outcome, Ctl* ctl, uint32_t entry_bytes, const uint32_t* in_off) {
  hipLaunchKernelGGL(k_measure_decide, dim3(1), dim3(1024), 0, st, part, cnt1, off, nblocks, nnz_in, nnz_out, u,
                     forced, rec, outcome, ctl, entry_bytes, in_off);
}

void launch_measure_write(hipStream_t st, bool wide, Buf in, Buf out, const uint64_t* nnz, uint32_t q,
                          const MeasRec* rec, const uint32_t* off, const uint32_t* in_off, int32_t q_next,
                          double2* part_next, uint32_t* cnt1_next, int grid) {
  if (wide)
    hipLaunchKernelGGL(k_measure_write<true>, dim3(grid), dim3(256), 0, st, in, out, nnz, q, rec, off, in_off, q_next,
                       part_next, cnt1_next);
  else
    hipLaunchKernelGGL(k_measure_write<false>, dim3(grid), dim3(256), 0, st, in, out, nnz, q, rec, off, in_off,
                       q_next, part_next, cnt1_next);
}

}  // namespace sparsesim

// ---------------------------------------------------------------------------
// Plain streaming copy (bandwidth reference for hardware byte counters).
namespace sparsesim {
namespace {
__global__ __launch_bounds__(256) void k_copy16(uint4* __restrict__ dst, const uint4* __restrict__ src, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
}  // namespace

void launch_copy16(hipStream_t st, void* dst, const void* src, uint64_t n16) {
  hipLaunchKernelGGL(k_copy16, dim3(8192), dim3(256), 0, st, static_cast<uint4*>(dst), static_cast<const uint4*>(src),
                     n16);
}
}  // namespace sparsesim
