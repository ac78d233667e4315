// Host check of the bit-sliced pass's op scheduling and packing: random plane
// ops are grouped by RunCompiler::group, then applied group by group with the
// kernel's group semantics (all reads of a group before its writes, shape
// bodies reading only their planes, TURN groups read-only) on random bit
// planes, and compared with applying the same ops one by one in their original
// order.  Built and run by test_bitslice_host.py; prints "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../paper_2105_01533_amd/csrc/run_compiler.h"

using namespace sparsesim;

namespace {

uint64_t sm_state;
uint64_t next_u64() {
  uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
uint32_t below(uint32_t n) { return (uint32_t)(next_u64() % n); }

constexpr int kWords = 4;   // independent 32-entry words per plane

struct State {
  std::vector<uint32_t> P;          // (nq + 2) planes x kWords
  std::vector<uint8_t> omega;       // per entry, mod 8
  std::vector<uint64_t> turns;      // per entry
  uint32_t& p(uint32_t q, int w) { return P[q * kWords + w]; }
};

// Sequential semantics of one BsOp.
void apply_seq(State& s, const BsOp& o, uint32_t nq) {
  for (int w = 0; w < kWords; ++w) {
    uint32_t cond = ~0u;
    for (int c = 0; c < o.nctrl; ++c) cond &= s.p(o.ctrl[c], w);
    if (o.op == kBsFlip) {
      s.p(o.target, w) ^= cond;
      continue;
    }
    const uint32_t x = cond & (o.cmode ? s.p(o.target, w) : ~0u);
    for (int j = 0; j < 32; ++j) {
      if (!((x >> j) & 1u)) continue;
      const size_t e = (size_t)w * 32 + j;
      if (o.op == kBsOmega) s.omega[e] = (uint8_t)((s.omega[e] + o.arg) & 7u);
      else s.turns[e] += o.arg;
    }
  }
  (void)nq;
}

// Field decoding of the packed kernel form.
uint32_t f_op(uint32_t a) { return a & 3u; }
uint32_t f_k(uint32_t a) { return (a >> 2) & 7u; }
uint32_t f_shape(uint32_t a0) { return (a0 >> 5) & 7u; }
uint32_t f_t(uint32_t a) { return (a >> 8) & 0xffu; }
uint32_t f_p0(uint32_t a) { return (a >> 16) & 0xffu; }
uint32_t f_p1(uint32_t a) { return a >> 24; }
uint32_t f_p2(uint32_t b) { return (b >> 8) & 0xffu; }

// Paired (or quad) flip or OMEGA groups: 8 (16) independent ops of one shape
// applied as one (all reads before all writes).
bool apply_multi(State& s, const BsGroup* G, int ng, uint32_t nq, std::string* why) {
  const uint32_t shape = f_shape(G[0].a[0]), scratch = nq + 1;
  for (int k = 1; k < ng; ++k) {
    if (G[k].a[1] & (kPairBit | kQuadBit)) return *why = "pair or quad flag inside a pair or quad", false;
    if (f_shape(G[k].a[0]) != shape) return *why = "mixed shapes in a pair or quad", false;
  }
  const int n = 4 * ng;
  uint32_t a[16], b[16];
  for (int k = 0; k < ng; ++k)
    for (int u = 0; u < 4; ++u) a[4 * k + u] = G[k].a[u], b[4 * k + u] = G[k].b[u];
  if (shape == kShapeOmega) {
    // Eighth-turn ops on their target bits: read-only, so any of them commute.
    for (int u = 0; u < n; ++u) {
      if (f_op(a[u]) != kBsOmega) return *why = "non-omega op in an OMEGA pair", false;
      if (f_p0(a[u]) != nq || f_p1(a[u]) != nq || f_p2(b[u]) != nq) return *why = "controlled op in an OMEGA pair", false;
    }
    for (int w = 0; w < kWords; ++w)
      for (int u = 0; u < n; ++u) {
        const uint32_t tv = s.p(f_t(a[u]), w);
        for (int j = 0; j < 32; ++j)
          if ((tv >> j) & 1u) s.omega[(size_t)w * 32 + j] = (uint8_t)((s.omega[(size_t)w * 32 + j] + f_k(a[u])) & 7u);
      }
    return true;
  }
  if (shape < kShapeX || shape > kShapeCCX) return *why = "bad pair shapes", false;
  for (int u = 0; u < n; ++u) {
    if (f_op(a[u]) != kBsFlip) return *why = "non-flip op in a pair", false;
    if (f_t(a[u]) == scratch) continue;
    for (int v = 0; v < n; ++v) {
      if (v == u) continue;
      const uint32_t r[3] = {f_t(a[v]), shape >= kShapeCX ? f_p0(a[v]) : 0xffffu, shape >= kShapeCCX ? f_p1(a[v]) : 0xffffu};
      for (uint32_t q : r)
        if (q == f_t(a[u])) return *why = "pair members conflict", false;
    }
  }
  for (int w = 0; w < kWords; ++w) {
    uint32_t tv[16], c[16];
    for (int u = 0; u < n; ++u) {
      tv[u] = s.p(f_t(a[u]), w);
      c[u] = (shape >= kShapeCX ? s.p(f_p0(a[u]), w) : ~0u) & (shape >= kShapeCCX ? s.p(f_p1(a[u]), w) : ~0u);
    }
    for (int u = 0; u < n; ++u) s.p(f_t(a[u]), w) = tv[u] ^ c[u];
  }
  return true;
}

bool apply_groups(State& s, const std::vector<BsGroup>& groups, uint32_t nq, std::string* why) {
  const uint32_t scratch = nq + 1;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const BsGroup& G = groups[gi];
    if (G.a[1] & kQuadBit) {
      if (G.a[1] & kPairBit) return *why = "pair and quad flags together", false;
      if (gi % 64 > 60) return *why = "quad across a batch of 64 groups", false;
      if (gi + 3 >= groups.size()) return *why = "quad without three more groups", false;
      if (!apply_multi(s, &groups[gi], 4, nq, why)) return false;
      gi += 3;
      continue;
    }
    if (G.a[1] & kPairBit) {
      if (gi % 64 == 63) return *why = "pair across a batch of 64 groups", false;
      if (gi + 1 >= groups.size()) return *why = "pair without a second group", false;
      if (!apply_multi(s, &groups[gi], 2, nq, why)) return false;
      ++gi;
      continue;
    }
    const uint32_t shape = f_shape(G.a[0]);
    const bool bare = (G.a[1] & kBareBit) != 0;
    if (bare) {
      // The kernel then reads only each op's target plane: every other
      // condition plane must be the all-ones plane.
      if (shape != kShapeTurn) return *why = "bare flag on a non-TURN group", false;
      for (int u = 0; u < kBsGroup; ++u)
        if (((G.a[u] >> 16) & 0xffu) != nq || ((G.a[u] >> 24) & 0xffu) != nq || ((G.b[u] >> 8) & 0xffu) != nq)
          return *why = "bare TURN group with a control plane", false;
    }
    for (int u = 1; u < kBsGroup; ++u)
      if (f_shape(G.a[u] & ~(u == 1 ? kBareBit : 0u))) return *why = "shape or pair bits set on a non-first op", false;
    // Independence: no member writes a plane another member reads or writes
    // (padding flips of the scratch plane excepted).
    for (int u = 0; u < kBsGroup; ++u) {
      const bool writes = f_op(G.a[u]) == kBsFlip && shape != kShapeTurn;
      if (!writes || f_t(G.a[u]) == scratch) continue;
      for (int v = 0; v < kBsGroup; ++v) {
        if (v == u) continue;
        const uint32_t r[4] = {f_t(G.a[v]), f_p0(G.a[v]), f_p1(G.a[v]), f_p2(G.b[v])};
        for (uint32_t q : r)
          if (q == f_t(G.a[u])) return *why = "group members conflict", false;
      }
    }
    for (int w = 0; w < kWords; ++w) {
      uint32_t tv[kBsGroup], c0[kBsGroup], c1[kBsGroup], c2[kBsGroup];
      for (int u = 0; u < kBsGroup; ++u) {   // every read before any write
        tv[u] = s.p(f_t(G.a[u]), w);
        c0[u] = shape == kShapeX || shape == kShapeOmega ? ~0u : s.p(f_p0(G.a[u]), w);
        c1[u] = shape == kShapeX || shape == kShapeCX || shape == kShapeOmega ? ~0u : s.p(f_p1(G.a[u]), w);
        c2[u] = shape == kShapeGeneric || shape == kShapePhase || shape == kShapeTurn ? s.p(f_p2(G.b[u]), w) : ~0u;
      }
      if (shape == kShapeOmega) {   // target-bit-only eighth turns; planes untouched
        for (int u = 0; u < kBsGroup; ++u) {
          if (f_op(G.a[u]) != kBsOmega) return *why = "non-omega op in an OMEGA group", false;
          if (f_p0(G.a[u]) != nq || f_p1(G.a[u]) != nq || f_p2(G.b[u]) != nq)
            return *why = "controlled op in an OMEGA group", false;
          for (int j = 0; j < 32; ++j)
            if ((tv[u] >> j) & 1u)
              s.omega[(size_t)w * 32 + j] = (uint8_t)((s.omega[(size_t)w * 32 + j] + f_k(G.a[u])) & 7u);
        }
        continue;
      }
      if (shape == kShapeTurn) {
        for (int u = 0; u < kBsGroup; ++u) {
          if (f_op(G.a[u]) != kBsTurn) return *why = "non-turn op in a TURN group", false;
          const uint32_t x = c0[u] & c1[u] & c2[u] & tv[u];
          for (int j = 0; j < 32; ++j)
            if ((x >> j) & 1u) s.turns[(size_t)w * 32 + j] += G.tau[u];
        }
        continue;
      }
      if (shape > kShapeOmega) return *why = "unknown shape", false;
      for (int u = 0; u < kBsGroup; ++u) {
        const uint32_t cond = c0[u] & c1[u] & c2[u];
        if (shape != kShapeGeneric && shape != kShapePhase && f_op(G.a[u]) != kBsFlip)
          return *why = "phase op in a flip-only group", false;
        if (f_op(G.a[u]) == kBsTurn) return *why = "turn op outside a TURN group", false;
        if (f_op(G.a[u]) == kBsFlip) s.p(f_t(G.a[u]), w) = tv[u] ^ cond;
        else s.p(f_t(G.a[u]), w) = tv[u];
        if (f_op(G.a[u]) == kBsOmega) {
          if (shape != kShapePhase) return *why = "phase op in a group without the PHASE shape", false;
          const uint32_t x = cond & tv[u];
          for (int j = 0; j < 32; ++j)
            if ((x >> j) & 1u)
              s.omega[(size_t)w * 32 + j] = (uint8_t)((s.omega[(size_t)w * 32 + j] + f_k(G.a[u])) & 7u);
        }
      }
    }
  }
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  const int cases = argc > 1 ? atoi(argv[1]) : 200;
  const uint32_t nqs[] = {4, 8, 17, 40, 64, 100, 128};
  size_t total_ops = 0, total_slots = 0;
  for (int c = 0; c < cases; ++c) {
    sm_state = 0x5EEDull * (c + 1);
    const uint32_t nq = nqs[c % 7];
    const uint32_t nops = 1 + below(c % 3 == 0 ? 40 : 600);
    RunCompiler rc;
    rc.n_qubits = nq;
    for (uint32_t i = 0; i < nops; ++i) {
      BsOp o{};
      const uint32_t kind = below(10);
      o.op = kind < 7 ? kBsFlip : kind < 9 ? kBsOmega : kBsTurn;
      const uint32_t maxc = nq - 1 < 3u ? nq - 1 : 3u;
      o.nctrl = (uint8_t)below(maxc + 1);
      // distinct target and controls
      uint32_t used[4];
      int nu = 0;
      while (nu < o.nctrl + 1) {
        const uint32_t q = below(nq);
        bool dup = false;
        for (int k = 0; k < nu; ++k) dup |= used[k] == q;
        if (!dup) used[nu++] = q;
      }
      o.target = (uint8_t)used[0];
      for (int k = 0; k < o.nctrl; ++k) o.ctrl[k] = (uint8_t)used[k + 1];
      o.cmode = o.op == kBsFlip ? 0 : (uint8_t)below(2);
      o.arg = o.op == kBsOmega ? 1 + below(7) : o.op == kBsTurn ? next_u64() | 1ull : 0;
      rc.ops.push_back(o);
    }
    rc.start = {0u, nops};
    std::vector<BsGroup> gops;
    BsRun br{};
    rc.group(0, 1, gops, &br);

    State ref, got;
    ref.P.resize((size_t)(nq + 2) * kWords);
    for (auto& v : ref.P) v = (uint32_t)next_u64();
    for (int w = 0; w < kWords; ++w) ref.p(nq, w) = ~0u;   // the all-ones plane
    ref.omega.assign(32 * kWords, 0);
    ref.turns.assign(32 * kWords, 0);
    got = ref;
    for (const BsOp& o : rc.ops) apply_seq(ref, o, nq);
    std::string why;
    if (!apply_groups(got, gops, nq, &why)) {
      printf("case %d (nq %u, ops %u): %s\n", c, nq, nops, why.c_str());
      return 1;
    }
    // Phase moved into the run constants by the rewrite of uncontrolled X
    // gates applies to every entry.
    for (auto& k : got.omega) k = (uint8_t)((k + br.g_omega) & 7u);
    for (auto& t : got.turns) t += br.g_turn;
    for (uint32_t q = 0; q <= nq; ++q)
      for (int w = 0; w < kWords; ++w)
        if (ref.p(q, w) != got.p(q, w)) {
          printf("case %d (nq %u, ops %u): plane %u differs\n", c, nq, nops, q);
          return 1;
        }
    if (ref.omega != got.omega || ref.turns != got.turns) {
      printf("case %d (nq %u, ops %u): phase accumulators differ\n", c, nq, nops);
      return 1;
    }
    total_ops += nops;
    total_slots += gops.size() * kBsGroup;
  }
  printf("OK cases=%d ops=%zu slots=%zu fill=%.3f\n", cases, total_ops, total_slots,
         (double)total_ops / (double)total_slots);
  return 0;
}
