// INT8-digit form of C = A B mod p on gfx950 (template; instantiated per
// digit count by mmp_int8_digits.hip).
//
// The paper's closing perspective proposes running the word products in a
// lower precision with more, narrower words.  Here each entry x of A and B
// (an integer in [0, p)) is written with D signed base-256 digits,
//     x' = sum_{i<D} 256^i d_i,   d_i in [-128, 127],   x' = x or x - p,
// so every digit plane is an int8 matrix.  The D^2 digit products run on the
// INT8 matrix cores with exact int32 accumulation; products with the same
// digit weight 256^s (i + j = s) share one accumulator, so there are 2D - 1
// accumulators per output.  A block of K k-terms keeps every accumulator
// exact when K times the extremes of one k-term's weight sum stay within
// int32; the planner takes those extremes over the digit vectors the entries
// can actually have (int8_bound_residues), at most D 2^14 in magnitude.
// After each block the accumulators are folded into a binary64 residue:
//     t = sum_s 256^s D_s mod p  (Horner's rule from the top weight down;
//         256 t is exact in binary64 and each step is reduced with Alg. 1's
//         quotient rounded to nearest, see fold_weights),
//     F = F + t mod p,
// and C = F is written once.  All binary64 steps follow Section 2.1.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "int8_digitize_kernel.h"
#include "mmp_internal.h"

namespace mmp {
namespace i8d {

typedef int int4v __attribute__((ext_vector_type(4)));

constexpr int kBK8 = 64;  // k-terms (bytes) per LDS stage: one 16x16x64 MFMA deep

__device__ __forceinline__ double fmod_full(double x, double p, double q) {
  const double c = floor(x * q);
  double d = fma(-c, p, x);
  d = (d >= p) ? d - p : d;
  d = (d < 0.0) ? d + p : d;
  return d;
}

// Horner's rule over the 2D - 1 digit weights: a value in [0, p) congruent
// to sum_s 256^s w[s], |w[s]| < 2^31.  Each step scales by 256 (exact: a
// power of two), reduces with Alg. 1's quotient rounded to nearest instead
// of floored (c = floor(fl(x q + 1/2)), no corrections), and adds the next
// weight.  With |x| < 2^61 the quotient estimate is within |x| 2^-52 / p of
// x / p + 1/2, so the reduced value stays within p/2 + 2^10 of zero and the
// sum with a weight stays below 2^53, exact.  One complete reduction ends it.
template <int ND>
__device__ __forceinline__ double fold_weights(const int (&w)[ND], double p, double q) {
  double t = (double)w[ND - 1];
#pragma unroll
  for (int s = ND - 2; s >= 0; s--) {
    const double x = 256.0 * t;
    const double c = floor(fma(x, q, 0.5));
    t = fma(-c, p, x) + (double)w[s];
  }
  return fmod_full(t, p, q);
}

__device__ __forceinline__ double addmod(double x, double y, double p) {
  const double s = x + y;
  return (s >= p) ? s - p : s;
}

struct GemmArgs {
  const int8_t* Ad;  // D planes of m x kp (16-row blocks, plane_at)
  const int8_t* Bd;  // D planes of n x kp
  double* C;
  int64_t m, n, kp, ldc;
  double p, q;
  int64_t stages_per_block;  // LDS stages (64 k-terms each) between folds
  int splits;                // split-K: k-ranges (1: none)
  double* partial;           // splits > 1: residues per k-range, [splits][m][n]
};

__device__ __forceinline__ void tile_coords(int bid, int nb, int nbm, int nbn, int& tmi, int& tni) {
  const int per = nb / 8, rem = nb % 8, xcd = bid % 8, loc = bid / 8;
  const int lin = (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
  const int group = 8 * nbn;
  const int gid = lin / group;
  const int first = gid * 8;
  const int gm = min(nbm - first, 8);
  const int in = lin - gid * group;
  tmi = first + in % gm;
  tni = in / gm;
}

struct GemmBatch {
  int njobs;
  int tile_start[kMaxBatch + 1];
  GemmArgs job[kMaxBatch];
};

// Workgroup shape per digit count.  WM x WN waves, each owning TM x TN
// 16x16 output tiles for all 2D - 1 digit weights; accumulator VGPRs per lane
// = (2D - 1) TM TN 4.  Two waves per SIMD hide the LDS and load latency, so
// every shape keeps a wave within 256 VGPRs: 4-wave groups (two groups per
// CU) up to 5 digits, one 8-wave group with narrower wave tiles beyond.
// NARROW (products with n <= 32): 64 x 32 tiles, so that no digit product
// is spent on padding columns; 16 x 32 wave tiles in 4-wave groups up to 5
// digits, 16 x 16 in an 8-wave group beyond.
template <int D, bool NARROW = false>
struct I8Shape {
  static constexpr int WM = NARROW ? 4 : 2;
  static constexpr int WN = NARROW ? (D <= 5 ? 1 : 2) : (D <= 5 ? 2 : 4);
  static constexpr int TM = NARROW ? 1 : 2;
  static constexpr int TN = NARROW ? (D <= 5 ? 2 : 1) : (D <= 5 ? 2 : 1);
  static constexpr int BM = WM * TM * 16;  // 64
  static constexpr int BN = WN * TN * 16;  // 64, or 32 when NARROW
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int GROUPS_PER_CU = D <= 5 ? 2 : 1;
  // LDS stages in the ring: three for the narrow tiles wherever the groups
  // per CU still fit (these products stream A's planes from HBM, and a
  // 64 x 32 stage computes in less time than one copy's latency), else two
  static constexpr int STAGES = (NARROW && D != 5) ? 3 : 2;
};

// Ring of NS LDS stages; each holds D digit planes of a BM x 64 slab of A
// and of a BN x 64 slab of B^T, 64 bytes per row with no padding (each 16-row
// part is one 1 KB block of a plane, copied by one instruction).  The four
// 16-byte chunks of row r are stored in the order q ^ f(r) with
// f(r) = ((r >> 2) ^ (r >> 1)) & 3.  An operand read takes chunk q of 16
// consecutive rows; f keeps those chunks in distinct banks whether the LDS
// serves 16 lanes over 256 bytes (distinct (r & 3, q ^ f)) or 8 lanes over
// 128 bytes (distinct (r & 1, q ^ f) within each 8 rows).
template <int D, int BM, int BN, int NS>
struct DigitRing {
  int8_t s[NS][D][BM + BN][64];
};

__device__ __forceinline__ int swz(int r, int q) { return ((q ^ (r >> 2) ^ (r >> 1)) & 3) * 16; }

// wait until at most N vector-memory operations of this wave are outstanding
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// The digit-product loop of one BM x BN tile.  Stage st + 1's slabs are
// copied from HBM straight into LDS (global_load_lds, one contiguous 1 KB
// block per wave instruction) while stage st is multiplied: all D^2 digit products on
// 16x16x64 INT8 MFMAs into the 2D - 1 digit-weight accumulators.  fold()
// runs after every stages_per_block stages and once at the end if the last
// block is partial.  Rows and columns past the matrix edge read an in-range
// row instead (their outputs are never stored); the k tail is zero in the
// planes.
template <int D, class S, class Fold>
__device__ __forceinline__ void digit_tile_loop(const int8_t* __restrict__ Ad, const int8_t* __restrict__ Bd,
                                                int64_t m, int64_t n, int64_t kp, int64_t m0, int64_t n0,
                                                int64_t st_begin, int64_t st_end,
                                                int64_t stages_per_block,
                                                DigitRing<D, S::BM, S::BN, S::STAGES>& sm,
                                                int4v (&acc)[2 * D - 1][S::TM][S::TN], Fold fold) {
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  constexpr int NW = S::WM * S::WN;
  constexpr int GROUPS = D * (BM + BN) / 16;  // 1 KB copy instructions per stage
  constexpr int IPW = (GROUPS + NW - 1) / NW;   // per wave; the last ones may idle
  static_assert(IPW < 64, "vmcnt range");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int64_t planeA = plane_size(m, kp), planeB = plane_size(n, kp);
  const int rl = lane >> 2;                       // row within a 16-row group
  const int ql = (lane & 3) ^ (((lane >> 4) ^ (lane >> 3)) & 3);  // chunk this lane copies: f(rl)

  // Copies move one 1 KB block (16 rows x 64 bytes) of a digit plane
  // straight into LDS (global_load_lds, 16 bytes a lane).  Each lane's byte
  // offset within its plane (row rl of the copy's 16, chunk ql; rows past m
  // or n read the last row instead, feeding outputs that are never stored)
  // is fixed for the whole loop; only the plane's scalar base moves, by one
  // block (1 KB) a stage.  The
  // wave index is made uniform once, so a copy's plane, base and LDS
  // destination are scalars and a stage's copies need no vector work.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  uint64_t voff[IPW];
#pragma unroll
  for (int e = 0; e < IPW; e++) {
    const int t = wv + NW * e;
    if (GROUPS % NW != 0 && t >= GROUPS) {
      voff[e] = 0;  // no copy
    } else if (t < D * BM / 16) {
      const int64_t row = m0 + 16 * (t % (BM / 16)) + rl;
      voff[e] = (uint64_t)plane_at(row < m ? row : m - 1, 16 * ql, kp);
    } else {
      const int64_t row = n0 + 16 * ((t - D * BM / 16) % (BN / 16)) + rl;
      voff[e] = (uint64_t)plane_at(row < n ? row : n - 1, 16 * ql, kp);
    }
  }
  // copies this wave issues per stage
  const int mine = (GROUPS % NW == 0 || wv < GROUPS % NW) ? IPW : IPW - 1;
  auto issue = [&](int64_t st, int b) {
#pragma unroll
    for (int e = 0; e < IPW; e++) {
      const int t = wv + NW * e;
      if (GROUPS % NW != 0 && t >= GROUPS) continue;  // uniform per wave
      const int8_t* base;
      int plane, row0;
      if (t < D * BM / 16) {
        plane = t / (BM / 16);
        row0 = 16 * (t % (BM / 16));
        base = Ad + plane * planeA + st * 1024;
      } else {
        const int t2 = t - D * BM / 16;
        plane = t2 / (BN / 16);
        row0 = BM + 16 * (t2 % (BN / 16));
        base = Bd + plane * planeB + st * 1024;
      }
      __builtin_amdgcn_global_load_lds((const void*)(base + voff[e]),
                                       (__attribute__((address_space(3))) void*)&sm.s[b][plane][row0][0], 16, 0, 0);
    }
  };

  constexpr int NS = S::STAGES;
  const int lrow = lane & 15, lq = lane >> 4;
  // the first NS - 1 stages in flight before the loop
#pragma unroll
  for (int i = 0; i < NS - 1; i++)
    if (st_begin + i < st_end) issue(st_begin + i, NS == 2 ? (int)((st_begin + i) & 1) : i);
  int64_t in_block = 0;
  int b3 = 0;  // three stages: buffer of stage st, (st - st_begin) mod 3
  for (int64_t st = st_begin; st < st_end; st++) {
    // two stages: buffer st & 1 (the prologue filled buffer st_begin & 1)
    const int b = NS == 2 ? (int)(st & 1) : b3;
    // This wave's copies of stage st are complete (with three stages, the
    // next stage's copies, issued after them, may still be in flight); the
    // barrier extends that to every wave and ends the reads of stage st - 1,
    // whose buffer the next copies overwrite.  A bare barrier: a fence here
    // would also wait for copies that may still be in flight; the empty asm
    // statements keep the compiler from moving LDS accesses or copies
    // across it.
    if (NS == 3 && st + 1 < st_end) {
      if (mine == IPW)
        wait_vm<IPW>();
      else
        wait_vm<(IPW > 0 ? IPW - 1 : 0)>();
    } else {
      wait_vm<0>();
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (st + NS - 1 < st_end) issue(st + NS - 1, NS == 2 ? (int)((st + 1) & 1) : (b == 0 ? NS - 1 : b - 1));
    int4v bf[D][TN];
#pragma unroll
    for (int j = 0; j < D; j++)
#pragma unroll
      for (int y = 0; y < TN; y++) {
        const int r = BM + wn + y * 16 + lrow;
        bf[j][y] = *(const int4v*)(&sm.s[b][j][r][swz(r, lq)]);
      }
#pragma unroll
    for (int i = 0; i < D; i++) {
      int4v af[TM];
#pragma unroll
      for (int x = 0; x < TM; x++) {
        const int r = wm + x * 16 + lrow;
        af[x] = *(const int4v*)(&sm.s[b][i][r][swz(r, lq)]);
      }
#pragma unroll
      for (int j = 0; j < D; j++)
#pragma unroll
        for (int x = 0; x < TM; x++)
#pragma unroll
          for (int y = 0; y < TN; y++)
            acc[i + j][x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[x], bf[j][y], acc[i + j][x][y], 0, 0, 0);
    }
    if (++in_block == stages_per_block) {
      in_block = 0;
      fold();
    }
    if (NS == 3) b3 = (b3 + 1 == NS) ? 0 : b3 + 1;
  }
  if (in_block != 0) fold();
}

template <int D, bool NARROW>
__global__ __launch_bounds__((I8Shape<D, NARROW>::THREADS), (I8Shape<D, NARROW>::GROUPS_PER_CU)) void
int8_digits_gemm_kernel(const GemmBatch bt) {
  using S = I8Shape<D, NARROW>;
  constexpr int ND = 2 * D - 1;
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  __shared__ __attribute__((aligned(1024))) DigitRing<D, BM, BN, S::STAGES> sm;

  int job = 0;
  while (job + 1 < bt.njobs && (int)blockIdx.x >= bt.tile_start[job + 1]) job++;
  const GemmArgs& a = bt.job[job];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int nbm = (int)((a.m + BM - 1) / BM), nbn = (int)((a.n + BN - 1) / BN);
  // split-K: the k-range varies fastest over workgroup ids.  Dispatch is
  // round-robin over the 8 XCDs, so with 8 (or 16, ...) k-ranges each XCD
  // works on its own k-range for every tile and reads that part of the
  // planes once into its L2, instead of every XCD reading all of A.
  const int bid = (int)blockIdx.x - bt.tile_start[job];
  const int split = a.splits > 1 ? bid % a.splits : 0;
  const int local_bid = a.splits > 1 ? bid / a.splits : bid;
  const int64_t nst = a.kp / kBK8, per_split = (nst + a.splits - 1) / a.splits;
  const int64_t st_begin = (int64_t)split * per_split;
  const int64_t st_end = st_begin + per_split < nst ? st_begin + per_split : nst;
  int tmi, tni;
  tile_coords(local_bid, nbm * nbn, nbm, nbn, tmi, tni);
  const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;

  int4v acc[ND][TM][TN];
#pragma unroll
  for (int s = 0; s < ND; s++)
#pragma unroll
    for (int x = 0; x < TM; x++)
#pragma unroll
      for (int y = 0; y < TN; y++) acc[s][x][y] = (int4v){0, 0, 0, 0};
  double F[TM][TN][4];
#pragma unroll
  for (int x = 0; x < TM; x++)
#pragma unroll
    for (int y = 0; y < TN; y++)
#pragma unroll
      for (int r = 0; r < 4; r++) F[x][y][r] = 0.0;

  const double p = a.p, q = a.q;
  // fold the digit-weight accumulators into the binary64 residues and clear them
  auto fold = [&]() {
#pragma unroll
    for (int x = 0; x < TM; x++)
#pragma unroll
      for (int y = 0; y < TN; y++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int w[ND];
#pragma unroll
          for (int s = 0; s < ND; s++) w[s] = acc[s][x][y][r];
          F[x][y][r] = addmod(F[x][y][r], fold_weights<ND>(w, p, q), p);
        }
#pragma unroll
    for (int s = 0; s < ND; s++)
#pragma unroll
      for (int x = 0; x < TM; x++)
#pragma unroll
        for (int y = 0; y < TN; y++) acc[s][x][y] = (int4v){0, 0, 0, 0};
  };
  digit_tile_loop<D, S>(a.Ad, a.Bd, a.m, a.n, a.kp, m0, n0, st_begin, st_end, a.stages_per_block, sm, acc, fold);

  // 16x16x64 INT8 MFMA output layout: D[i][j] is value (i & 3) of lane j + 16 (i >> 2).
  const int lrow = lane & 15;
#pragma unroll
  for (int x = 0; x < TM; x++)
#pragma unroll
    for (int y = 0; y < TN; y++) {
      const int64_t col = n0 + wn + y * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t row = m0 + wm + x * 16 + (lane >> 4) * 4 + r;
        if (row < a.m && col < a.n) {
          if (a.splits == 1)  // C is written once: a streaming store
            __builtin_nontemporal_store(F[x][y][r] + 0.0, &a.C[row * a.ldc + col]);
          else
            a.partial[((int64_t)split * a.m + row) * a.n + col] = F[x][y][r];
        }
      }
    }
}

}  // namespace i8d
}  // namespace mmp
