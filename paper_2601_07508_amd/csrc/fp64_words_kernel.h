// Fused FP64-word kernel for C = A B mod p on gfx950 (template; instantiated
// per word pair by mmp_fp64_words.hip).
//
// One workgroup computes a BM x BN tile of C for all u v word pairs at once:
//   1. prologue per LDS stage: coalesced global loads of an A (BM x KR) and a
//      B (KR x BN) slab; every entry is split into words (Section 3.1, Alg. 4)
//      on the way into LDS, so word planes never exist in HBM;
//   2. hot loop: for every word pair (i, j), 16x16x4 FP64 MFMAs accumulate
//      A_i B_j into VGPR accumulators; after each k-block of at most the
//      paper's block size (Section 2.2, Prop. blockProduct; Section 3.2,
//      Prop. UVMW) every accumulator is reduced mod p with the fma-based
//      reduction (Section 2.1, Alg. 1);
//   3. epilogue: a complete reduction, then the word products are recombined
//      as sum_i alpha^i sum_j beta^j T_ij mod p by Horner's rule, each step a
//      modular product by alpha or beta (Section 2.1, Alg. 2) and a modular
//      addition; C is written once.
//
// Exactness in the MFMA: operands are integers, every partial sum of a block
// is an integer of magnitude at most 2^53 (the block-size bound), so the
// order in which the matrix core adds the products does not matter.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mmp_internal.h"

namespace mmp {
namespace fp64w {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 waves of 64
constexpr int kPadA = 1;       // A plane rows: kBK + 1 doubles (16 rows hit distinct banks)
constexpr int kPadB = 16;      // B plane rows: BN + 16 doubles (adjacent k-slots 32 banks apart)

// ---- scalar modular arithmetic (binary64, explicit fma, no reassociation)

// Alg. 1 without its two corrections, optionally biased by K p (with K = 1/2
// the quotient is rounded to nearest and d lies within p/2 + 3 of zero, the
// centered words' range):
// c = floor(fl(x q + K)) is within one of floor(x / p) + K (the quotient
// estimate of Prop. fpModularReductionFMA's proof, with the error of one
// more rounding of a value below 2^(t+1) / p), so d = x - c p lies in
// [-K p - p, -K p + 2p) for any integer |x| <= 2^t.  K = 0 gives [-p, 2p);
// K = floor(2^t / p) - 1 gives [-2^t, -2^t + 4p), the bottom of the exact
// range.  fma(x, q, 0) is the plain product x q.
__device__ __forceinline__ double fmod_lazy(double x, double p, double q, double bias) {
  const double c = floor(fma(x, q, bias));
  return fma(-c, p, x);
}

// Alg. 1 complete: result in [0, p).
__device__ __forceinline__ double fmod_full(double x, double p, double q) {
  const double c = floor(x * q);
  double d = fma(-c, p, x);
  d = (d >= p) ? d - p : d;
  d = (d < 0.0) ? d + p : d;
  return d;
}

// Alg. 2: x y mod p via the error-free product h + l = x y.
__device__ __forceinline__ double mulmod(double x, double y, double p, double q) {
  const double h = x * y;
  const double l = fma(x, y, -h);
  const double c = floor(h * q);
  const double d = fma(-c, p, h);
  double e = d + l;
  e = (e >= p) ? e - p : e;
  e = (e < 0.0) ? e + p : e;
  return e;
}

__device__ __forceinline__ double addmod(double x, double y, double p) {
  const double s = x + y;
  return (s >= p) ? s - p : s;
}

// Alg. 4 on one entry: words w[0..W-1] with x = sum_i a^i w[i], 0 <= w[i] < a.
// The quotient is floor(T / a) with a correctly rounded division (Lemma
// exactFpDiv); when a is a power of two, T * (1/a) is the same exact value.
template <int W>
__device__ __forceinline__ void split_words(double x, double a, double ainv, double (&w)[W]) {
  double t = x;
#pragma unroll
  for (int i = 0; i < W - 1; i++) {
    const double r = (ainv != 0.0) ? floor(t * ainv) : floor(t / a);
    w[i] = fma(-a, r, t);
    t = r;
  }
  w[W - 1] = t;
}

// Centered words (the library's variant of Alg. 4): x in [0, p) is first
// taken to x - p when 2x > p, then split with quotients rounded to nearest,
// so x - (0 or p) = sum_i a^i w[i] with |w[i]| <= a/2 + 1 below the top
// word.  The words are congruent-preserving: the recombination is unchanged.
template <int W>
__device__ __forceinline__ void split_words_centered(double x, double p, double a, double ainv, double (&w)[W]) {
  double t = (x + x > p) ? x - p : x;
#pragma unroll
  for (int i = 0; i < W - 1; i++) {
    const double r = (ainv != 0.0) ? rint(t * ainv) : rint(t / a);
    w[i] = fma(-a, r, t);
    t = r;
  }
  w[W - 1] = t;
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
// that consecutive tile numbers run on the same XCD (shared L2), then walk
// tiles in groups of 8 tile-rows so neighbours share A and B panels.
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

// s_waitcnt lgkmcnt(0) alone: this wave's LDS writes are complete, while its
// global loads (vmcnt) may stay in flight across the barrier that follows.
__device__ __forceinline__ void wait_lds_writes() {
  __builtin_amdgcn_s_waitcnt(0xF | (0x3 << 14) | (0x7 << 4) | (0x0 << 8));
}

// Workgroup barrier that does not wait for outstanding global loads (the
// compiler's __syncthreads would add vmcnt(0) and end the prefetch).  The
// empty asm statements keep the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  wait_lds_writes();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int U, int V, int TM, int TN, int FE>
__global__ __launch_bounds__(kThreads, 2) void fp64_words_kernel(const Fp64Batch bt) {
  static_assert(FE == 1 || FE == 2 || FE == 4, "reduction period");
  // which product of the batch this workgroup belongs to (uniform, scalar)
  int job = 0;
  while (job + 1 < bt.njobs && (int)blockIdx.x >= bt.tile_start[job + 1]) job++;
  const Fp64Args& a = bt.job[job];
  // split-K: tiles of one k-range are consecutive; split index major
  const int tiles = (int)(((a.m + 2 * TM * 16 - 1) / (2 * TM * 16)) * ((a.n + 2 * TN * 16 - 1) / (2 * TN * 16)));
  const int split = ((int)blockIdx.x - bt.tile_start[job]) / tiles;
  const int local_bid = ((int)blockIdx.x - bt.tile_start[job]) - split * tiles;
  constexpr int BM = 2 * TM * 16;
  constexpr int BN = 2 * TN * 16;
  constexpr int LDA = kBK + kPadA;
  constexpr int LDB = BN + kPadB;
  constexpr int NA = (BM * kBK + kThreads - 1) / kThreads;  // A slab entries per thread (max)
  constexpr int NB = (kBK * BN + kThreads - 1) / kThreads;
  // two LDS stages: stage s is multiplied from buffer s & 1 while stage
  // s + 1 is written into the other
  __shared__ double As[2][U][BM][LDA];
  __shared__ double Bs[2][V][kBK][LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * TM * 16;
  const int wn = (wave & 1) * TN * 16;

  const int nbm = (int)((a.m + BM - 1) / BM);
  const int nbn = (int)((a.n + BN - 1) / BN);
  int tmi, tni;
  tile_coords(local_bid, nbm * nbn, nbm, nbn, tmi, tni);
  const int64_t m0 = (int64_t)tmi * BM;
  const int64_t n0 = (int64_t)tni * BN;

  // zero both buffers once: slots that no k-term maps to stay zero
  for (int i = tid; i < 2 * U * BM * LDA; i += kThreads) (&As[0][0][0][0])[i] = 0.0;
  for (int i = tid; i < 2 * V * kBK * LDB; i += kThreads) (&Bs[0][0][0][0])[i] = 0.0;

  // Per-thread slab positions, fixed for every stage.  Real k-term kk of a
  // stage lands in slot (kk / L) S + kk % L when a block fits in a stage
  // (S <= kBK, the remaining S - L slots of each block stay zero), else in
  // slot kk (blocks span whole stages, L = S).
  const int KR = a.KR;
  // packed positions: A: row << 16 | kk << 8 | slot;  B: kk << 16 | col << 8 | slot;  -1: idle
  int a_pos[NA], b_pos[NB];
#pragma unroll
  for (int e = 0; e < NA; e++) {
    const int idx = tid + e * kThreads;
    const int r = idx / KR, kk = idx - r * KR;
    const int slot = (a.S <= kBK) ? (kk / a.L) * a.S + kk % a.L : kk;
    a_pos[e] = (idx < BM * KR) ? ((r << 16) | (kk << 8) | slot) : -1;
  }
#pragma unroll
  for (int e = 0; e < NB; e++) {
    const int idx = tid + e * kThreads;
    const int kk = idx / BN, c = idx % BN;
    const int slot = (a.S <= kBK) ? (kk / a.L) * a.S + kk % a.L : kk;
    b_pos[e] = (idx < KR * BN) ? ((kk << 16) | (c << 8) | slot) : -1;
  }

  double ra[NA], rb[NB];
  auto load_stage = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < NA; e++) {
      const int pos = a_pos[e];
      const int64_t row = m0 + (pos >> 16), col = k0 + ((pos >> 8) & 0xff);
      ra[e] = (pos >= 0 && row < a.m && col < a.k) ? a.A[row * a.lda + col] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; e++) {
      const int pos = b_pos[e];
      const int64_t row = k0 + (pos >> 16), col = n0 + ((pos >> 8) & 0xff);
      rb[e] = (pos >= 0 && row < a.k && col < a.n) ? a.B[row * a.ldb + col] : 0.0;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; e++) {
      const int pos = a_pos[e];
      if (pos >= 0) {
        double w[U];
        if (a.centered)
          split_words_centered<U>(ra[e], a.p, a.alpha, a.ainv, w);
        else
          split_words<U>(ra[e], a.alpha, a.ainv, w);
#pragma unroll
        for (int i = 0; i < U; i++) As[buf][i][pos >> 16][pos & 0xff] = w[i];
      }
    }
#pragma unroll
    for (int e = 0; e < NB; e++) {
      const int pos = b_pos[e];
      if (pos >= 0) {
        double w[V];
        if (a.centered)
          split_words_centered<V>(rb[e], a.p, a.beta, a.binv, w);
        else
          split_words<V>(rb[e], a.beta, a.binv, w);
#pragma unroll
        for (int j = 0; j < V; j++) Bs[buf][j][pos & 0xff][(pos >> 8) & 0xff] = w[j];
      }
    }
  };

  d4 acc[U][V][TM][TN];
#pragma unroll
  for (int i = 0; i < U; i++)
#pragma unroll
    for (int j = 0; j < V; j++)
#pragma unroll
      for (int x = 0; x < TM; x++)
#pragma unroll
        for (int y = 0; y < TN; y++) acc[i][j][x][y] = (d4){a.acc_init, a.acc_init, a.acc_init, a.acc_init};

  const double p = a.p, q = a.q, bias = a.bias;
  const int64_t nstages_all = (a.k + KR - 1) / KR;
  // this split's stages: [s_begin, s_end)
  const int64_t per_split = (nstages_all + a.splits - 1) / a.splits;
  const int64_t s_begin = (int64_t)split * per_split;
  const int64_t s_end = s_begin + per_split < nstages_all ? s_begin + per_split : nstages_all;
  const int lrow = lane & 15, lk = lane >> 4;

  // In-loop reduction of every accumulator (Alg. 1).  The correction-free
  // form leaves values in [-p, 2p); when the planner could not show that a
  // block started there stays within 2^t, the two corrections follow.
  auto reduce_all = [&]() {
#pragma unroll
    for (int i = 0; i < U; i++)
#pragma unroll
      for (int j = 0; j < V; j++)
#pragma unroll
        for (int x = 0; x < TM; x++)
#pragma unroll
          for (int y = 0; y < TN; y++)
#pragma unroll
            for (int r = 0; r < 4; r++) acc[i][j][x][y][r] = fmod_lazy(acc[i][j][x][y][r], p, q, bias);
    if (!a.lazy) {
#pragma unroll
      for (int i = 0; i < U; i++)
#pragma unroll
        for (int j = 0; j < V; j++)
#pragma unroll
          for (int x = 0; x < TM; x++)
#pragma unroll
            for (int y = 0; y < TN; y++)
#pragma unroll
              for (int r = 0; r < 4; r++) {
                double d = acc[i][j][x][y][r];
                d = (d >= p) ? d - p : d;
                acc[i][j][x][y][r] = (d < 0.0) ? d + p : d;
              }
    }
  };

  // Stage s is split into buffer (s - s_begin) & 1 one iteration ahead; its
  // global loads are issued one further iteration ahead, so they are in
  // flight during a whole stage of MFMAs.  One barrier per stage: after it,
  // every wave has finished reading the buffer the next store overwrites.
  int stage_in_block = 0;
  __syncthreads();  // the zeroed buffers are visible before any store
  if (s_begin < s_end) {
    load_stage(s_begin * KR);
    store_stage(0);
    if (s_begin + 1 < s_end) load_stage((s_begin + 1) * KR);
  }
  lds_barrier();
  for (int64_t s = s_begin; s < s_end; s++) {
    const int buf = (int)((s - s_begin) & 1);
#pragma unroll
    for (int ks = 0; ks < kBK / 4; ks++) {
      double af[U][TM], bf[V][TN];
#pragma unroll
      for (int i = 0; i < U; i++)
#pragma unroll
        for (int x = 0; x < TM; x++) af[i][x] = As[buf][i][wm + x * 16 + lrow][ks * 4 + lk];
#pragma unroll
      for (int j = 0; j < V; j++)
#pragma unroll
        for (int y = 0; y < TN; y++) bf[j][y] = Bs[buf][j][ks * 4 + lk][wn + y * 16 + lrow];
#pragma unroll
      for (int i = 0; i < U; i++)
#pragma unroll
        for (int j = 0; j < V; j++)
#pragma unroll
          for (int x = 0; x < TM; x++)
#pragma unroll
            for (int y = 0; y < TN; y++)
              acc[i][j][x][y] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][x], bf[j][y], acc[i][j][x][y], 0, 0, 0);
      if constexpr (FE < 4) {
        if ((ks + 1) % FE == 0) reduce_all();
      }
    }
    if constexpr (FE == 4) {
      if (++stage_in_block == a.stages_per_block) {
        stage_in_block = 0;
        reduce_all();
      }
    }
    if (s + 1 < s_end) {
      store_stage(buf ^ 1);
      if (s + 2 < s_end) load_stage((s + 2) * KR);
    }
    lds_barrier();
  }

  // Epilogue: complete reduction and Horner recombination, then one store.
  // 16x16x4 FP64 MFMA output layout: D[i][j] is value (i >> 2) of lane j + 16 (i & 3).
#pragma unroll
  for (int x = 0; x < TM; x++) {
#pragma unroll
    for (int y = 0; y < TN; y++) {
      const int64_t col = n0 + wn + y * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t row = m0 + wm + x * 16 + lk + 4 * r;
        double c = 0.0;
#pragma unroll
        for (int i = U - 1; i >= 0; i--) {
          double si = fmod_full(acc[i][V - 1][x][y][r], p, q);
#pragma unroll
          for (int j = V - 2; j >= 0; j--)
            si = addmod(mulmod(a.beta, si, p, q), fmod_full(acc[i][j][x][y][r], p, q), p);
          c = (i == U - 1) ? si : addmod(mulmod(a.alpha, c, p, q), si, p);
        }
        if (row < a.m && col < a.n) {
          if (a.splits == 1)
            a.C[row * a.ldc + col] = c + 0.0;  // +0.0: canonical zero
          else
            a.partial[((int64_t)split * a.m + row) * a.n + col] = c;  // residue of this k-range
        }
      }
    }
  }
}

// The tile shapes of fp64_tile_c() as compile-time constants.
template <int UV, int ID>
struct TileOf {
  static constexpr int tm = fp64_tile_c(ID, UV).tm;
  static constexpr int tn = fp64_tile_c(ID, UV).tn;
};

// Tiles of one product for a given shape.
template <int BM, int BN>
inline int64_t tiles_of(const Fp64Args& a) {
  return ((a.m + BM - 1) / BM) * ((a.n + BN - 1) / BN) * a.splits;
}

template <int U, int V, int ID, int FE>
int launch_shape(const Fp64Batch& b0, hipStream_t s) {
  constexpr int TM = TileOf<U * V, ID>::tm, TN = TileOf<U * V, ID>::tn;
  constexpr int BM = 2 * 16 * TM, BN = 2 * 16 * TN;
  Fp64Batch b = b0;
  int64_t total = 0;
  for (int j = 0; j < b.njobs; j++) {
    b.tile_start[j] = (int)total;
    total += tiles_of<BM, BN>(b.job[j]);
    if (total > 0x7fffffff) return (int)hipErrorInvalidValue;
  }
  b.tile_start[b.njobs] = (int)total;
  if (total <= 0) return 0;
  TimerTok* t = timer_begin("fp64_words");
  hipExtLaunchKernelGGL((fp64_words_kernel<U, V, TM, TN, FE>), dim3((unsigned)total), dim3(kThreads), 0, s,
                        timer_start(t), timer_stop(t), 0, b);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

}  // namespace fp64w
}  // namespace mmp
