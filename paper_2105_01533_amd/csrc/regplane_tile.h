// Register-plane form of the fused phase/permutation pass (Sec. 3.2), for
// gfx950 (device code; included by mono_regplane.hip).
//
// A wave owns a tile of 2048 entries: lane l holds entries l + 64 j, j =
// 0..31, as 32-bit bit-planes (bit j of plane q = qubit q of entry j).  The
// planes live in VGPRs v100 .. v100 + nq + 2 for the whole run: the compiler
// is capped below v80 (amdgpu_num_vgpr), so it never allocates v80 and above,
// and only the inline assembly here touches them.  A gate names its planes by
// index at run time, so the plane registers are addressed with the GPR
// indexing mode (s_set_gpr_idx_on / _idx: the index, the low byte of an SGPR,
// is added to the register number of the instruction's src0 and, when
// enabled, its vdst).  A CNOT on the tile is then three scalar and two vector
// instructions, with no LDS round trip and no dependent-latency chain.
//
// Register map (fixed, assembly only):
//   v80        P  -- eighth-turn accumulator, weight 4 (one bit per entry)
//   v81, v82   Q  -- weight-2 counter, 2 bits
//   v83..v85   R  -- weight-1 counter, 3 bits
//   v86, v87   temporaries; v88 load address; v89 = 16 x lane
//   v90..v93   the program chunk in use, v94..v97 the next one
//   v100 + q   plane q; plane nq is all ones, nq + 1 scratch, nq + 2 zero.
// An eighth-turn op adding k where x holds adds x (k & 1) to R, x ((k >> 1) &
// 1) to Q and x (k >> 2) to P, so the entry's count is R + 2 Q + 4 P mod 8.
//
// The program (RpRec quads, see sim_internal.h) is read 64 quads (1 KiB) at a
// time with one vector load per lane (lane l holds quad l in v90..v93), the
// next chunk always in flight, and broadcast with v_readlane: no scalar-cache
// latency on the path.  Flip and eighth-turn segments run in one assembly
// loop that reads each segment header and dispatches on its shape; turn and
// general eighth-turn segments return to C++, which reads their quads through
// the same chunk registers.  Arbitrary-angle phases (TURN) accumulate exact
// 64-bit turn fractions per entry in LDS through a 16-entry subset-sum table
// per group of four ops.
#pragma once
#include "sim_internal.h"

namespace sparsesim {
namespace rp {

// Highest VGPR the kernel reserves for planes (v100..v230: up to 131 planes).
// The kernel declares it clobbered whatever a run's plane count, so its
// allocation is 231 VGPRs and at most two waves share a SIMD.  Narrower
// allocations (132 and 164 VGPRs, three waves per SIMD) gave results on
// multi-million-entry states that differed from run to run, as did two waves
// of different programs on one SIMD; waves of one program at most two per
// SIMD reproduce the LDS-plane pass bit for bit (the launcher keeps passes
// apart).  The 132-register form also loaded a label's second word
// (v132..v163) past its allocation.
constexpr uint32_t kVmax = 230;
constexpr uint32_t kTurnAccBytes = 32 * 64 * 8;   // per wave: 32 entries x 64 lanes x 64-bit turns

// LSB-first 32x32 bit transpose (out[q] bit j = in[j] bit q), by the
// recursive block-swap method of Warren, Hacker's Delight, Sec. 7-3: five
// rounds of masked swaps of 16-, 8-, 4-, 2- and 1-bit blocks.
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

// omega^k = e^{i pi k / 4}, exact.
__device__ __forceinline__ double2 omega_pow(uint32_t k) {
  const double h = 0.70710678118654752440;
  const double x = (k & 1u) ? h : 1.0, y = (k & 1u) ? h : 0.0;
  const uint32_t r = (k >> 1) & 3u;
  const double re = r == 0 ? x : (r == 1 ? -y : (r == 2 ? -x : y));
  const double im = r == 0 ? y : (r == 1 ? x : (r == 2 ? -y : -x));
  return make_double2(re, im);
}

// Plane q (the low byte of a wave-uniform value) into a compiler register,
// and back.
__device__ __forceinline__ uint32_t rd_plane(uint32_t q) {
  uint32_t r;
  asm volatile(
      "s_set_gpr_idx_on %1, gpr_idx(SRC0)\n\t"
      "v_mov_b32 %0, v100\n\t"
      "s_set_gpr_idx_off"
      : "=v"(r)
      : "s"(q)
      : "m0");
  return r;
}
__device__ __forceinline__ void wr_plane(uint32_t q, uint32_t v) {
  asm volatile(
      "s_set_gpr_idx_on %0, gpr_idx(DST)\n\t"
      "v_mov_b32 v100, %1\n\t"
      "s_set_gpr_idx_off" ::"s"(q),
      "v"(v)
      : "m0");
}

#define RP_IN(R, X) asm volatile("v_mov_b32 v" #R ", %0" ::"v"(X))
#define RP_OUT(R, X) asm volatile("v_mov_b32 %0, v" #R : "=v"(X))
#define RP_IN_WORD0(a) \
  RP_IN(100, a[0]); RP_IN(101, a[1]); RP_IN(102, a[2]); RP_IN(103, a[3]); RP_IN(104, a[4]); RP_IN(105, a[5]); RP_IN(106, a[6]); RP_IN(107, a[7]); \
  RP_IN(108, a[8]); RP_IN(109, a[9]); RP_IN(110, a[10]); RP_IN(111, a[11]); RP_IN(112, a[12]); RP_IN(113, a[13]); RP_IN(114, a[14]); RP_IN(115, a[15]); \
  RP_IN(116, a[16]); RP_IN(117, a[17]); RP_IN(118, a[18]); RP_IN(119, a[19]); RP_IN(120, a[20]); RP_IN(121, a[21]); RP_IN(122, a[22]); RP_IN(123, a[23]); \
  RP_IN(124, a[24]); RP_IN(125, a[25]); RP_IN(126, a[26]); RP_IN(127, a[27]); RP_IN(128, a[28]); RP_IN(129, a[29]); RP_IN(130, a[30]); RP_IN(131, a[31]);
#define RP_OUT_WORD0(a) \
  RP_OUT(100, a[0]); RP_OUT(101, a[1]); RP_OUT(102, a[2]); RP_OUT(103, a[3]); RP_OUT(104, a[4]); RP_OUT(105, a[5]); RP_OUT(106, a[6]); RP_OUT(107, a[7]); \
  RP_OUT(108, a[8]); RP_OUT(109, a[9]); RP_OUT(110, a[10]); RP_OUT(111, a[11]); RP_OUT(112, a[12]); RP_OUT(113, a[13]); RP_OUT(114, a[14]); RP_OUT(115, a[15]); \
  RP_OUT(116, a[16]); RP_OUT(117, a[17]); RP_OUT(118, a[18]); RP_OUT(119, a[19]); RP_OUT(120, a[20]); RP_OUT(121, a[21]); RP_OUT(122, a[22]); RP_OUT(123, a[23]); \
  RP_OUT(124, a[24]); RP_OUT(125, a[25]); RP_OUT(126, a[26]); RP_OUT(127, a[27]); RP_OUT(128, a[28]); RP_OUT(129, a[29]); RP_OUT(130, a[30]); RP_OUT(131, a[31]);
#define RP_IN_WORD1(a) \
  RP_IN(132, a[0]); RP_IN(133, a[1]); RP_IN(134, a[2]); RP_IN(135, a[3]); RP_IN(136, a[4]); RP_IN(137, a[5]); RP_IN(138, a[6]); RP_IN(139, a[7]); \
  RP_IN(140, a[8]); RP_IN(141, a[9]); RP_IN(142, a[10]); RP_IN(143, a[11]); RP_IN(144, a[12]); RP_IN(145, a[13]); RP_IN(146, a[14]); RP_IN(147, a[15]); \
  RP_IN(148, a[16]); RP_IN(149, a[17]); RP_IN(150, a[18]); RP_IN(151, a[19]); RP_IN(152, a[20]); RP_IN(153, a[21]); RP_IN(154, a[22]); RP_IN(155, a[23]); \
  RP_IN(156, a[24]); RP_IN(157, a[25]); RP_IN(158, a[26]); RP_IN(159, a[27]); RP_IN(160, a[28]); RP_IN(161, a[29]); RP_IN(162, a[30]); RP_IN(163, a[31]);
#define RP_OUT_WORD1(a) \
  RP_OUT(132, a[0]); RP_OUT(133, a[1]); RP_OUT(134, a[2]); RP_OUT(135, a[3]); RP_OUT(136, a[4]); RP_OUT(137, a[5]); RP_OUT(138, a[6]); RP_OUT(139, a[7]); \
  RP_OUT(140, a[8]); RP_OUT(141, a[9]); RP_OUT(142, a[10]); RP_OUT(143, a[11]); RP_OUT(144, a[12]); RP_OUT(145, a[13]); RP_OUT(146, a[14]); RP_OUT(147, a[15]); \
  RP_OUT(148, a[16]); RP_OUT(149, a[17]); RP_OUT(150, a[18]); RP_OUT(151, a[19]); RP_OUT(152, a[20]); RP_OUT(153, a[21]); RP_OUT(154, a[22]); RP_OUT(155, a[23]); \
  RP_OUT(156, a[24]); RP_OUT(157, a[25]); RP_OUT(158, a[26]); RP_OUT(159, a[27]); RP_OUT(160, a[28]); RP_OUT(161, a[29]); RP_OUT(162, a[30]); RP_OUT(163, a[31]);
#define RP_IN_WORD2(a) \
  RP_IN(164, a[0]); RP_IN(165, a[1]); RP_IN(166, a[2]); RP_IN(167, a[3]); RP_IN(168, a[4]); RP_IN(169, a[5]); RP_IN(170, a[6]); RP_IN(171, a[7]); \
  RP_IN(172, a[8]); RP_IN(173, a[9]); RP_IN(174, a[10]); RP_IN(175, a[11]); RP_IN(176, a[12]); RP_IN(177, a[13]); RP_IN(178, a[14]); RP_IN(179, a[15]); \
  RP_IN(180, a[16]); RP_IN(181, a[17]); RP_IN(182, a[18]); RP_IN(183, a[19]); RP_IN(184, a[20]); RP_IN(185, a[21]); RP_IN(186, a[22]); RP_IN(187, a[23]); \
  RP_IN(188, a[24]); RP_IN(189, a[25]); RP_IN(190, a[26]); RP_IN(191, a[27]); RP_IN(192, a[28]); RP_IN(193, a[29]); RP_IN(194, a[30]); RP_IN(195, a[31]);
#define RP_OUT_WORD2(a) \
  RP_OUT(164, a[0]); RP_OUT(165, a[1]); RP_OUT(166, a[2]); RP_OUT(167, a[3]); RP_OUT(168, a[4]); RP_OUT(169, a[5]); RP_OUT(170, a[6]); RP_OUT(171, a[7]); \
  RP_OUT(172, a[8]); RP_OUT(173, a[9]); RP_OUT(174, a[10]); RP_OUT(175, a[11]); RP_OUT(176, a[12]); RP_OUT(177, a[13]); RP_OUT(178, a[14]); RP_OUT(179, a[15]); \
  RP_OUT(180, a[16]); RP_OUT(181, a[17]); RP_OUT(182, a[18]); RP_OUT(183, a[19]); RP_OUT(184, a[20]); RP_OUT(185, a[21]); RP_OUT(186, a[22]); RP_OUT(187, a[23]); \
  RP_OUT(188, a[24]); RP_OUT(189, a[25]); RP_OUT(190, a[26]); RP_OUT(191, a[27]); RP_OUT(192, a[28]); RP_OUT(193, a[29]); RP_OUT(194, a[30]); RP_OUT(195, a[31]);
#define RP_IN_WORD3(a) \
  RP_IN(196, a[0]); RP_IN(197, a[1]); RP_IN(198, a[2]); RP_IN(199, a[3]); RP_IN(200, a[4]); RP_IN(201, a[5]); RP_IN(202, a[6]); RP_IN(203, a[7]); \
  RP_IN(204, a[8]); RP_IN(205, a[9]); RP_IN(206, a[10]); RP_IN(207, a[11]); RP_IN(208, a[12]); RP_IN(209, a[13]); RP_IN(210, a[14]); RP_IN(211, a[15]); \
  RP_IN(212, a[16]); RP_IN(213, a[17]); RP_IN(214, a[18]); RP_IN(215, a[19]); RP_IN(216, a[20]); RP_IN(217, a[21]); RP_IN(218, a[22]); RP_IN(219, a[23]); \
  RP_IN(220, a[24]); RP_IN(221, a[25]); RP_IN(222, a[26]); RP_IN(223, a[27]); RP_IN(224, a[28]); RP_IN(225, a[29]); RP_IN(226, a[30]); RP_IN(227, a[31]);
#define RP_OUT_WORD3(a) \
  RP_OUT(196, a[0]); RP_OUT(197, a[1]); RP_OUT(198, a[2]); RP_OUT(199, a[3]); RP_OUT(200, a[4]); RP_OUT(201, a[5]); RP_OUT(202, a[6]); RP_OUT(203, a[7]); \
  RP_OUT(204, a[8]); RP_OUT(205, a[9]); RP_OUT(206, a[10]); RP_OUT(207, a[11]); RP_OUT(208, a[12]); RP_OUT(209, a[13]); RP_OUT(210, a[14]); RP_OUT(211, a[15]); \
  RP_OUT(212, a[16]); RP_OUT(213, a[17]); RP_OUT(214, a[18]); RP_OUT(215, a[19]); RP_OUT(216, a[20]); RP_OUT(217, a[21]); RP_OUT(218, a[22]); RP_OUT(219, a[23]); \
  RP_OUT(220, a[24]); RP_OUT(221, a[25]); RP_OUT(222, a[26]); RP_OUT(223, a[27]); RP_OUT(224, a[28]); RP_OUT(225, a[29]); RP_OUT(226, a[30]); RP_OUT(227, a[31]);

// Raw buffer resource over n bytes at p (gfx9 descriptor word 3): loads past
// n return zero and stores past n are dropped, so a ragged tile needs no
// per-entry branches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)n, 0x00020000);
}
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4i buf_rsrc_v4(const void* p, uint32_t n) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  v4i r;
  r.x = (int)(uint32_t)a;
  r.y = (int)(uint32_t)(a >> 32);   // stride 0
  r.z = (int)n;
  r.w = 0x00020000;
  return r;
}

// ---- program fetch -----------------------------------------------------------
// Next quad: the four words of quad `lane` of the current chunk, then advance;
// past the chunk's last quad the prefetched chunk becomes current and the one
// after it is requested (at byte offset off of the program, then off += 1 KiB).
// The program resource returns zeros past its end: an END header.
#define RP_NEXTQ                                  \
  "s_add_u32 %[lane], %[lane], 1\n\t"             \
  "s_cmp_eq_u32 %[lane], 64\n\t"                  \
  "s_cbranch_scc0 8f\n\t"                         \
  "s_waitcnt vmcnt(0)\n\t"                        \
  "v_mov_b32 v90, v94\n\t"                        \
  "v_mov_b32 v91, v95\n\t"                        \
  "v_mov_b32 v92, v96\n\t"                        \
  "v_mov_b32 v93, v97\n\t"                        \
  "v_add_u32 v88, %[off], v89\n\t"                \
  "buffer_load_dwordx4 v[94:97], v88, %[rs], 0 offen\n\t" \
  "s_add_u32 %[off], %[off], 1024\n\t"            \
  "s_mov_b32 %[lane], 0\n"                        \
  "8:\n\t"
// Read a quad into s92..s95 (GPR indexing must be off: v_readlane's source is
// a VGPR operand).
#define RP_READQ                                  \
  "s_set_gpr_idx_off\n\t"                         \
  "v_readlane_b32 s92, v90, %[lane]\n\t"          \
  "v_readlane_b32 s93, v91, %[lane]\n\t"          \
  "v_readlane_b32 s94, v92, %[lane]\n\t"          \
  "v_readlane_b32 s95, v93, %[lane]\n\t" RP_NEXTQ

// ---- op bodies -------------------------------------------------------------
// Op words: t | c0 << 8 | c1 << 16 | c2 << 24 (flips), t (eighth turns).
// s_set_gpr_idx_* use the low byte of the named SGPR as the plane index, so
// a right shift by 8 k selects field k.
#define RP_F1(W)                                  \
  "s_lshr_b32 s96, " W ", 8\n\t"                  \
  "s_set_gpr_idx_on s96, gpr_idx(SRC0)\n\t"       \
  "v_mov_b32 v86, v100\n\t"                       \
  "s_set_gpr_idx_on " W ", gpr_idx(SRC0,DST)\n\t" \
  "v_xor_b32 v100, v100, v86\n\t"
#define RP_F2(W)                                  \
  "s_lshr_b32 s96, " W ", 8\n\t"                  \
  "s_lshr_b32 s97, " W ", 16\n\t"                 \
  "s_set_gpr_idx_on s96, gpr_idx(SRC0)\n\t"       \
  "v_mov_b32 v86, v100\n\t"                       \
  "s_set_gpr_idx_idx s97\n\t"                     \
  "v_and_b32 v86, v100, v86\n\t"                  \
  "s_set_gpr_idx_on " W ", gpr_idx(SRC0,DST)\n\t" \
  "v_xor_b32 v100, v100, v86\n\t"
#define RP_F3(W)                                  \
  "s_lshr_b32 s96, " W ", 8\n\t"                  \
  "s_lshr_b32 s97, " W ", 16\n\t"                 \
  "s_set_gpr_idx_on s96, gpr_idx(SRC0)\n\t"       \
  "v_mov_b32 v86, v100\n\t"                       \
  "s_set_gpr_idx_idx s97\n\t"                     \
  "v_and_b32 v86, v100, v86\n\t"                  \
  "s_lshr_b32 s97, " W ", 24\n\t"                 \
  "s_set_gpr_idx_idx s97\n\t"                     \
  "v_and_b32 v86, v100, v86\n\t"                  \
  "s_set_gpr_idx_on " W ", gpr_idx(SRC0,DST)\n\t" \
  "v_xor_b32 v100, v100, v86\n\t"
// Eighth-turn adds of x = plane t (v100 under SRC0 indexing).  bitop3 truth
// tables index bits as S0 * 4 + S1 * 2 + S2: 0x6a = S2 ^ (S0 & S1), 0x78 =
// S0 ^ (S1 & S2).
#define RP_ADD_P "v_xor_b32 v80, v100, v80\n\t"
#define RP_ADD_Q "v_bitop3_b32 v82, v100, v81, v82 bitop3:0x6a\n\tv_xor_b32 v81, v100, v81\n\t"
#define RP_ADD_R1 "v_and_b32 v86, v100, v83\n\tv_xor_b32 v83, v100, v83\n\t"
#define RP_ADD_R2 "s_set_gpr_idx_off\n\tv_bitop3_b32 v85, v85, v84, v86 bitop3:0x78\n\tv_xor_b32 v84, v84, v86\n\t"
#define RP_ON(W) "s_set_gpr_idx_on " W ", gpr_idx(SRC0)\n\t"
#define RP_OB1(W) RP_ON(W) RP_ADD_R1 RP_ADD_R2
#define RP_OB2(W) RP_ON(W) RP_ADD_Q
#define RP_OB3(W) RP_ON(W) RP_ADD_R1 RP_ADD_Q RP_ADD_R2
#define RP_OB4(W) RP_ON(W) RP_ADD_P
#define RP_OB5(W) RP_ON(W) RP_ADD_R1 RP_ADD_P RP_ADD_R2
#define RP_OB6(W) RP_ON(W) RP_ADD_Q RP_ADD_P
#define RP_OB7(W) RP_ON(W) RP_ADD_R1 RP_ADD_Q RP_ADD_P RP_ADD_R2

// A segment loop at label L: each quad is four ops of one shape; count
// quads, then back to the header reader (label 20).
#define RP_SEG(L, OP)                             \
  #L ":\n\t" RP_READQ OP("s92") OP("s93") OP("s94") OP("s95") \
  "s_sub_u32 %[cnt], %[cnt], 1\n\t"               \
  "s_cmp_eq_u32 %[cnt], 0\n\t"                    \
  "s_cbranch_scc0 " #L "b\n\t"                    \
  "s_branch 20b\n"
#define RP_CASE(SHAPE, L) "s_cmp_eq_u32 %[shape], " #SHAPE "\n\ts_cbranch_scc1 " #L "f\n\t"

// The interpreter: header quads (w0 = shape | quads << 8) and the segments of
// flips and eighth turns, until a header of another shape (returned in shape,
// with cnt) is read.
#define RP_INTERP                                 \
  "20:\n\t"                                       \
  "s_set_gpr_idx_off\n\t"                         \
  "v_readlane_b32 s92, v90, %[lane]\n\t" RP_NEXTQ \
  "s_and_b32 %[shape], s92, 0xff\n\t"             \
  "s_lshr_b32 %[cnt], s92, 8\n\t"                 \
  RP_CASE(1, 21) RP_CASE(2, 22) RP_CASE(3, 23)    \
  RP_CASE(9, 31) RP_CASE(10, 32) RP_CASE(11, 33) RP_CASE(12, 34) RP_CASE(13, 35) RP_CASE(14, 36) RP_CASE(15, 37) \
  "s_branch 40f\n"                                \
  RP_SEG(21, RP_F1) RP_SEG(22, RP_F2) RP_SEG(23, RP_F3)                  \
  RP_SEG(31, RP_OB1) RP_SEG(32, RP_OB2) RP_SEG(33, RP_OB3) RP_SEG(34, RP_OB4) \
  RP_SEG(35, RP_OB5) RP_SEG(36, RP_OB6) RP_SEG(37, RP_OB7)             \
  "40:\n\t"                                       \
  "s_set_gpr_idx_off"

struct Fetch {
  uint32_t lane, off;
  v4i rs;
};

// Load chunks 0 and 1 of the program; v89 = 16 x lane.
__device__ __forceinline__ void fetch_start(Fetch& f, const RpRec* prog, uint32_t nrec, int lane) {
  f.rs = buf_rsrc_v4(prog, 16u * nrec);
  f.lane = 0;
  f.off = 2048;
  asm volatile(
      "v_lshlrev_b32 v89, 4, %[id]\n\t"
      "buffer_load_dwordx4 v[90:93], v89, %[rs], 0 offen\n\t"
      "v_add_u32 v88, 1024, v89\n\t"
      "buffer_load_dwordx4 v[94:97], v88, %[rs], 0 offen\n\t"
      "s_waitcnt vmcnt(0)" ::[id] "v"(lane),
      [rs] "s"(f.rs)
      : "memory");
}

__device__ __forceinline__ void next_quad(Fetch& f, uint32_t (&w)[4]) {
  asm volatile(
      "s_set_gpr_idx_off\n\t"
      "v_readlane_b32 %[w0], v90, %[lane]\n\t"
      "v_readlane_b32 %[w1], v91, %[lane]\n\t"
      "v_readlane_b32 %[w2], v92, %[lane]\n\t"
      "v_readlane_b32 %[w3], v93, %[lane]\n\t" RP_NEXTQ
      : [w0] "=&s"(w[0]), [w1] "=&s"(w[1]), [w2] "=&s"(w[2]), [w3] "=&s"(w[3]), [lane] "+s"(f.lane),
        [off] "+s"(f.off)
      : [rs] "s"(f.rs)
      : "m0", "scc", "memory");
}

// General eighth-turn ops, two per quad (cond word, k): x = planes t & c0 &
// c1 & c2, then the weighted adds with k's bits as masks.
__device__ __forceinline__ void omega_general(Fetch& f, uint32_t nquads) {
  for (uint32_t i = 0; i < nquads; ++i) {
    uint32_t w[4];
    next_quad(f, w);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t c = w[2 * h], k = w[2 * h + 1];
      const uint32_t x = rd_plane(c) & rd_plane(c >> 8) & rd_plane(c >> 16) & rd_plane(c >> 24);
      const uint32_t m1 = (k & 1u) ? ~0u : 0u, m2 = (k & 2u) ? ~0u : 0u, m4 = (k & 4u) ? ~0u : 0u;
      asm volatile(
          "v_bitop3_b32 v80, %0, %3, v80 bitop3:0x6a\n\t"   // P ^= x & m4
          "v_and_b32 v86, %2, %0\n\t"
          "v_bitop3_b32 v82, v82, v81, v86 bitop3:0x78\n\t" // Q += x & m2
          "v_xor_b32 v81, v81, v86\n\t"
          "v_and_b32 v86, %1, %0\n\t"
          "v_and_b32 v87, v83, v86\n\t"                      // R += x & m1
          "v_xor_b32 v83, v83, v86\n\t"
          "v_bitop3_b32 v85, v85, v84, v87 bitop3:0x78\n\t"
          "v_xor_b32 v84, v84, v87" ::"v"(x),
          "s"(m1), "s"(m2), "s"(m4));
    }
  }
}

// TURN groups: three quads per group of four ops (cond words; fractions of
// ops 0, 1; of ops 2, 3).  Each entry's accumulator (LDS, acc[64 j + lane])
// gains the sum of the fractions of the ops whose condition holds for it: per
// group, one of 16 subset sums, kept in a 16-entry LDS table and read with
// one 64-bit load per entry.  C groups share one read-modify-write of the
// accumulators (C tables side by side), which is what bounds the pass on
// LDS bandwidth.
template <bool BARE, int C>
__device__ __forceinline__ void turn_chunk(Fetch& f, uint64_t* acc, uint64_t* table, int lane) {
  uint32_t B[C][8];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    uint32_t cw[4], t01[4], t23[4];
    next_quad(f, cw);
    next_quad(f, t01);
    next_quad(f, t23);
    uint32_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = rd_plane(cw[u]);
      if (!BARE) x[u] &= rd_plane(cw[u] >> 8) & rd_plane(cw[u] >> 16) & rd_plane(cw[u] >> 24);
    }
    const uint64_t tau[4] = {((uint64_t)t01[1] << 32) | t01[0], ((uint64_t)t01[3] << 32) | t01[2],
                             ((uint64_t)t23[1] << 32) | t23[0], ((uint64_t)t23[3] << 32) | t23[2]};
    // Entry j's offset in table c, 8 x (the ops, bit u = op u, whose
    // condition holds for it), is byte j >> 3 of B[c][j & 7]: bit j of x[u]
    // moves to bit 8 (j >> 3) + 3 + u by one constant shift; the four merge
    // under disjoint byte-lane masks.
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      uint32_t v = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int sh = w - 3 - u;
        const uint32_t y = sh >= 0 ? x[u] >> sh : x[u] << -sh;
        v |= y & (0x01010101u << (3 + u));
      }
      B[c][w] = v;
    }
    // Table entry m (lane m < 16) is the sum of the fractions named by m's
    // bits.  (The lane number is made opaque here so that the four masks are
    // formed where they are used, not kept live across the whole tile.)
    int l = lane;
    asm volatile("" : "+v"(l));
    uint64_t S = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) S += tau[u] & (0ull - (uint64_t)((l >> u) & 1));
    if (l < 16) table[16 * c + l] = S;   // the wave's LDS accesses complete in order
    __builtin_amdgcn_sched_barrier(0);  // one group's planes at a time
  }
  const char* tb = reinterpret_cast<const char*>(table);
#pragma unroll
  for (int j0 = 0; j0 < 32; j0 += 4) {
    uint64_t a[4], v[C][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = j0 + k;
      a[k] = acc[64 * j + lane];
#pragma unroll
      for (int c = 0; c < C; ++c)
        v[c][k] = *reinterpret_cast<const uint64_t*>(tb + 128 * c + __builtin_amdgcn_ubfe(B[c][j & 7], 8 * (j >> 3), 8));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint64_t t = a[k];
#pragma unroll
      for (int c = 0; c < C; ++c) t += v[c][k];
      acc[64 * (j0 + k) + lane] = t;
    }
    // Keep the blocks apart (otherwise every entry's table address is formed
    // up front, and they do not fit the registers).
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <bool BARE>
__device__ __forceinline__ void turn_groups(Fetch& f, uint32_t ng, uint64_t* acc, uint64_t* table, int lane) {
  uint32_t g = 0;
  for (; g + 2 <= ng; g += 2) turn_chunk<BARE, 2>(f, acc, table, lane);
  if (g < ng) turn_chunk<BARE, 1>(f, acc, table, lane);
}

// Labels of the tile (word w of each label: bits 32w..32w+31) into planes.
__device__ __forceinline__ void load_word(const Buf& b, uint64_t base, uint32_t lim, int w, int lane) {
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc((w < 2 ? b.key_lo : b.key_hi) + base, 8 * lim);
  const int off = 8 * lane + 4 * (w & 1);
  uint32_t a[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) a[j] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 512 * j, 0);
  transpose32(a);
  if (w == 0) { RP_IN_WORD0(a) }
  else if (w == 1) { RP_IN_WORD1(a) }
  else if (w == 2) { RP_IN_WORD2(a) }
  else { RP_IN_WORD3(a) }
}

__device__ __forceinline__ void store_word(const Buf& b, uint64_t base, uint32_t lim, int w, int nq, int lane) {
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc((w < 2 ? b.key_lo : b.key_hi) + base, 8 * lim);
  const int off = 8 * lane + 4 * (w & 1);
  uint32_t a[32];
  if (w == 0) { RP_OUT_WORD0(a) }
  else if (w == 1) { RP_OUT_WORD1(a) }
  else if (w == 2) { RP_OUT_WORD2(a) }
  else { RP_OUT_WORD3(a) }
  // Planes at and above nq are the all-ones, scratch and zero planes (or
  // unused): labels have no such bits.
#pragma unroll
  for (int q = 0; q < 32; ++q) a[q] = 32 * w + q < nq ? a[q] : 0u;
  transpose32(a);
#pragma unroll
  for (int j = 0; j < 32; ++j) __builtin_amdgcn_raw_buffer_store_b32(a[j], rs, off, 512 * j, 0);
}

// Apply a run's program (nrec records) to the tile at base (lim valid
// entries).  TURNS: the kernel provides acc, the wave's turn accumulators in
// LDS, and table, its subset-sum tables; a run uses them if it has turn ops
// (the result does not depend on TURNS otherwise).
template <bool TURNS>
__device__ __forceinline__ void rp_tile(const Buf& b, uint64_t base, uint32_t lim, const RpRec* prog, uint32_t nrec,
                                        const BsRun& run, uint64_t* acc, uint64_t* table) {
  // The lane number, opaque to the optimizer: values derived from it are
  // formed where used, not kept live across a kernel's loop over tiles.
  int lane = threadIdx.x;
  asm volatile("" : "+v"(lane));
  const uint32_t nq = run.n_planes;
  const bool turns = TURNS && run.has_turns;
  const uint32_t rw = run.words_read | run.words_write;
  Fetch f;
  fetch_start(f, prog, nrec, lane);
#pragma unroll
  for (int w = 0; w < 4; ++w)
    if (rw & (1u << w)) load_word(b, base, lim, w, lane);
  wr_plane(nq, ~0u);       // all ones
  wr_plane(nq + 2, 0u);    // zero
  asm volatile(
      "v_mov_b32 v80, 0\n\tv_mov_b32 v81, 0\n\tv_mov_b32 v82, 0\n\t"
      "v_mov_b32 v83, 0\n\tv_mov_b32 v84, 0\n\tv_mov_b32 v85, 0");
  if (turns) {
#pragma unroll
    for (int j = 0; j < 32; ++j) acc[64 * j + lane] = 0;
  }
  for (;;) {
    uint32_t shape, cnt;
    asm volatile(RP_INTERP
                 : [lane] "+s"(f.lane), [off] "+s"(f.off), [shape] "=&s"(shape), [cnt] "=&s"(cnt)
                 : [rs] "s"(f.rs)
                 : "s92", "s93", "s94", "s95", "s96", "s97", "m0", "scc", "memory");
    if (shape == kRpOG) {
      omega_general(f, cnt);
    } else if (shape == kRpTB || shape == kRpTG) {
      if (turns) {
        if (shape == kRpTB) turn_groups<true>(f, cnt, acc, table, lane);
        else turn_groups<false>(f, cnt, acc, table, lane);
      } else {
        break;   // the host never sends turn ops to this variant
      }
    } else {
      break;   // END (zero words past the program) or an unknown shape
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the last prefetch
  // Labels back to memory (only words some gate flips).
#pragma unroll
  for (int w = 0; w < 4; ++w)
    if (run.words_write & (1u << w)) store_word(b, base, lim, w, (int)nq, lane);
  if (!run.has_phase) return;
  uint32_t P, Q0, Q1, R0, R1, R2;
  asm volatile(
      "v_mov_b32 %0, v80\n\tv_mov_b32 %1, v81\n\tv_mov_b32 %2, v82\n\t"
      "v_mov_b32 %3, v83\n\tv_mov_b32 %4, v84\n\tv_mov_b32 %5, v85"
      : "=v"(P), "=v"(Q0), "=v"(Q1), "=v"(R0), "=v"(R1), "=v"(R2));
  // One complex multiply per amplitude by the accumulated phase.
  double2* amp = b.amp + base + lane;
#pragma unroll 1
  for (int j = 0; j < 32; ++j) {
    if (64u * j + lane >= lim) break;
    const uint32_t rj = ((R0 >> j) & 1u) | (((R1 >> j) & 1u) << 1) | (((R2 >> j) & 1u) << 2);
    const uint32_t qj = ((Q0 >> j) & 1u) | (((Q1 >> j) & 1u) << 1);
    const uint32_t k = (rj + 2u * qj + 4u * ((P >> j) & 1u) + run.g_omega) & 7u;
    double2 f2;
    if (!turns && run.g_turn == 0) {
      f2 = omega_pow(k);
    } else {
      const uint64_t tj = turns ? acc[64 * j + lane] : 0ull;
      const uint64_t T = tj + run.g_turn + ((uint64_t)k << 61);
      double sn, cs;
      sincospi((double)(T >> 11) * 0x1p-52, &sn, &cs);   // angle = 2 pi T / 2^64
      f2 = make_double2(cs, sn);
    }
    amp[64 * j] = cmul(amp[64 * j], f2);
  }
}

}  // namespace rp
}  // namespace sparsesim
