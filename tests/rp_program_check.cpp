// Host check of the register-plane pass's programs (RunCompiler::schedule):
// random phase/permutation op lists are scheduled into segments, replayed with
// the kernel's segment semantics on random bit planes (flip quads in order,
// eighth-turn ops split by the bits of k into the weight-1, -2 and -4
// accumulators, turn groups through their fractions), and compared with
// applying the same ops one by one in their original order.  Also checks the
// program's layout: header words, counts, planes in range, and padding ops
// that change nothing.  Built and run by test_bitslice_host.py; prints "OK" on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
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
  std::vector<uint32_t> P;          // (nq + 3) planes x kWords
  std::vector<uint8_t> omega;       // per entry, mod 8
  std::vector<uint64_t> turns;      // per entry
  uint32_t& p(uint32_t q, int w) { return P[q * kWords + w]; }
};

void apply_seq(State& s, const BsOp& o) {
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
}

// Replay a program with the kernel's semantics.  Weighted accumulators as in
// the kernel: R (weight 1), Q (weight 2), P (weight 4), per entry mod 8.
bool replay(State& s, const std::vector<RpRec>& prog, uint32_t nq, std::string* why) {
  const uint32_t np = nq + 3, scratch = nq + 1;
  std::vector<uint8_t> R(32 * kWords, 0), Q(32 * kWords, 0), Pw(32 * kWords, 0);
  auto add = [&](int w, uint32_t x, uint32_t k) {
    for (int j = 0; j < 32; ++j) {
      if (!((x >> j) & 1u)) continue;
      const size_t e = (size_t)w * 32 + j;
      if (k & 1u) R[e] = (uint8_t)((R[e] + 1) & 7u);
      if (k & 2u) Q[e] = (uint8_t)((Q[e] + 1) & 3u);
      if (k & 4u) Pw[e] ^= 1u;
    }
  };
  auto plane_ok = [&](uint32_t q) { return q < np; };
  auto cond = [&](uint32_t c, int w) {
    return s.p(c & 0xff, w) & s.p((c >> 8) & 0xff, w) & s.p((c >> 16) & 0xff, w) & s.p(c >> 24, w);
  };
  size_t pc = 0;
  for (;;) {
    if (pc >= prog.size()) break;   // past the end the kernel reads zeros: END
    const RpRec& h = prog[pc];
    const uint32_t shape = h.w[0] & 0xff, cnt = h.w[0] >> 8;
    if (h.w[1] || h.w[2] || h.w[3]) return *why = "header words 1..3 not zero", false;
    if (shape == kRpEnd) return *why = "END header inside the program", false;
    if (cnt == 0) return *why = "empty segment", false;
    const size_t body = pc + 1;
    const size_t len = (shape == kRpTB || shape == kRpTG) ? 3 * (size_t)cnt : cnt;
    if (body + len > prog.size()) return *why = "segment runs past the program", false;
    for (size_t r = 0; r < len; ++r) {
      const RpRec& q = prog[body + r];
      if (shape >= kRpF1 && shape <= kRpF3) {
        for (int u = 0; u < 4; ++u) {
          const uint32_t wd = q.w[u], t = wd & 0xff;
          uint32_t cs[3] = {(wd >> 8) & 0xff, (wd >> 16) & 0xff, wd >> 24};
          if (!plane_ok(t)) return *why = "plane out of range", false;
          for (uint32_t c = 0; c < shape; ++c)
            if (!plane_ok(cs[c])) return *why = "plane out of range", false;
          if (t == nq || t == nq + 2) return *why = "flip of the all-ones or zero plane", false;
          for (int w = 0; w < kWords; ++w) {
            uint32_t c = ~0u;
            for (uint32_t k = 0; k < shape; ++k) c &= s.p(cs[k], w);
            if (t == scratch) continue;   // padding only
            s.p(t, w) ^= c;
          }
        }
      } else if (shape > kRpOB && shape < kRpOB + 8) {
        for (int u = 0; u < 4; ++u) {
          if (q.w[u] >= np) return *why = "bad OB word", false;
          for (int w = 0; w < kWords; ++w) add(w, s.p(q.w[u], w), shape - kRpOB);
        }
      } else if (shape == kRpOG) {
        for (int h2 = 0; h2 < 2; ++h2) {
          const uint32_t c = q.w[2 * h2], k = q.w[2 * h2 + 1];
          for (int b = 0; b < 4; ++b)
            if (!plane_ok((c >> (8 * b)) & 0xff)) return *why = "plane out of range", false;
          if (k > 7) return *why = "bad OG k", false;
          for (int w = 0; w < kWords; ++w) add(w, cond(c, w), k);
        }
      } else if (shape == kRpTB || shape == kRpTG) {
        const RpRec* g = &prog[body + r];
        const uint64_t tau[4] = {((uint64_t)g[1].w[1] << 32) | g[1].w[0], ((uint64_t)g[1].w[3] << 32) | g[1].w[2],
                                 ((uint64_t)g[2].w[1] << 32) | g[2].w[0], ((uint64_t)g[2].w[3] << 32) | g[2].w[2]};
        for (int u = 0; u < 4; ++u) {
          const uint32_t c = g[0].w[u];
          for (int b = 0; b < 4; ++b)
            if (!plane_ok((c >> (8 * b)) & 0xff)) return *why = "plane out of range", false;
          for (int w = 0; w < kWords; ++w) {
            const uint32_t x = shape == kRpTB ? s.p(c & 0xff, w) : cond(c, w);
            for (int j = 0; j < 32; ++j)
              if ((x >> j) & 1u) s.turns[(size_t)w * 32 + j] += tau[u];
          }
        }
        r += 2;
      } else {
        return *why = "unknown shape", false;
      }
    }
    pc = body + len;
  }
  for (size_t e = 0; e < s.omega.size(); ++e) s.omega[e] = (uint8_t)((s.omega[e] + R[e] + 2 * Q[e] + 4 * Pw[e]) & 7u);
  for (int w = 0; w < kWords; ++w)
    if (s.p(nq + 2, w) != 0u || s.p(nq, w) != ~0u) return *why = "all-ones or zero plane changed", false;
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  const int cases = argc > 1 ? atoi(argv[1]) : 200;
  const uint32_t nqs[] = {4, 8, 17, 29, 40, 64, 100, 125};
  size_t total_ops = 0, total_rec = 0, total_seg = 0;
  for (int c = 0; c < cases; ++c) {
    sm_state = 0xA11CEull * (c + 1);
    const uint32_t nq = nqs[c % 8];
    const uint32_t nops = 1 + below(c % 3 == 0 ? 40 : (c % 5 == 0 ? 6000 : 600));
    RunCompiler rc;
    rc.n_qubits = nq;
    for (uint32_t i = 0; i < nops; ++i) {
      BsOp o{};
      const uint32_t kind = below(10);
      o.op = kind < 7 ? kBsFlip : kind < 9 ? kBsOmega : kBsTurn;
      const uint32_t maxc = nq - 1 < 3u ? nq - 1 : 3u;
      o.nctrl = (uint8_t)below(maxc + 1);
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
    std::vector<RpRec> prog;
    BsRun br{};
    rc.schedule(0, 1, prog, &br);
    if (prog.size() > RunCompiler::rp_records_bound(nops, nq)) {
      printf("case %d (nq %u, ops %u): %zu records exceed the bound\n", c, nq, nops, prog.size());
      return 1;
    }
    State ref, got;
    ref.P.resize((size_t)(nq + 3) * kWords);
    for (auto& v : ref.P) v = (uint32_t)next_u64();
    for (int w = 0; w < kWords; ++w) {
      ref.p(nq, w) = ~0u;       // all ones
      ref.p(nq + 2, w) = 0u;    // zero
    }
    ref.omega.assign(32 * kWords, 0);
    ref.turns.assign(32 * kWords, 0);
    got = ref;
    for (const BsOp& o : rc.ops) apply_seq(ref, o);
    std::string why;
    if (!replay(got, prog, nq, &why)) {
      printf("case %d (nq %u, ops %u): %s\n", c, nq, nops, why.c_str());
      return 1;
    }
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
    size_t seg = 0;
    for (size_t pc = 0; pc < prog.size();) {
      const uint32_t sh = prog[pc].w[0] & 0xff, cnt = prog[pc].w[0] >> 8;
      ++seg;
      pc += 1 + ((sh == kRpTB || sh == kRpTG) ? 3 * (size_t)cnt : cnt);
    }
    total_ops += nops;
    total_rec += prog.size();
    total_seg += seg;
  }
  printf("OK cases=%d ops=%zu quads=%zu segments=%zu ops/segment=%.2f\n", cases, total_ops, total_rec, total_seg,
         (double)total_ops / (double)total_seg);
  return 0;
}
