// Fused FP64-word kernel for C = A B mod p on gfx950 (template; instantiated
// per word pair by mmp_fp64_words.hip).
//
// One workgroup computes a BM x BN tile of C for all u v word pairs at once:
//   1. per LDS stage (16 k-slots): buffer loads of an A (BM x KR) and a B
//      (KR x BN) slab, issued a stage ahead into registers; every entry is
//      split into words (Section 3.1, Alg. 4, or the centered variant) on the
//      way into one of two LDS buffers, so word planes never exist in HBM;
//   2. hot loop: for every word pair (i, j), 16x16x4 FP64 MFMAs accumulate
//      A_i B_j into VGPR accumulators; after each k-block of at most the
//      block size (the paper's: Section 2.2, Prop. blockProduct; Section 3.2,
//      Prop. UVMW; or an opt-in bound) every accumulator is reduced mod p
//      with the fma-based reduction (Section 2.1, Alg. 1);
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
#include <type_traits>

#include "mmp_internal.h"

namespace mmp {
namespace fp64w {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 waves of 64
constexpr int kPadA = 1;       // A plane rows: kBK + 1 doubles (16 rows hit distinct banks)
// B plane rows hold BN doubles with no padding; odd k-slots store column c
// at c ^ 16, so the two k-slots one half-wave reads sit 32 banks apart.
__device__ __forceinline__ int bswz(int slot, int c) { return c ^ ((slot & 1) << 4); }

// Raw buffer loads (dword 3 of the resource for the gfx9 family): reads at or
// past the resource's byte count return zero instead of touching memory.
constexpr int kBufferWord3 = 0x00020000;
// A byte offset past every resource the kernel builds (their byte counts are
// clamped to 2^31 - 1): a load from it returns zero.
constexpr uint32_t kIdleOffset = 0xFFFFFFF0u;
__device__ __forceinline__ double buffer_load_f64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  typedef int v2i __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

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

// Alg. 4 on one entry, with the library's centered variant.
//   paper words (CEN = false): x = sum_i a^i w[i] with 0 <= w[i] < a; each
//     quotient is floor(t / a): r = floor(fl(t ainv)) with ainv = fl(1/a) is
//     exact when a is a power of two and otherwise within one of the
//     quotient (t < 2^53), so one correction step in each direction makes it
//     exact (fix = 1);
//   centered words (CEN = true): x is first taken to x - p when
//     2x > p, and r = floor(fl(t ainv + 1/2)) rounds to nearest within
//     |t| 2^-52 < 1/2, so |w[i]| < a/2 + 1 below the top word with no
//     correction; x - (0 or p) = sum_i a^i w[i] exactly either way.
// Branch-free: fix is uniform over the launch; CEN is a template argument
// (the caller branches once per stage), so paper words pay nothing for it.
template <int W, bool CEN>
__device__ __forceinline__ void split_entry(double x, double p, double a, double ainv, bool fix, double (&w)[W]) {
  constexpr double rbias = CEN ? 0.5 : 0.0;
  double t = (CEN && x + x > p) ? x - p : x;
#pragma unroll
  for (int i = 0; i < W - 1; i++) {
    double r = floor(fma(t, ainv, rbias));
    double d = fma(-a, r, t);
    if (!CEN && fix) {
      const bool lo = d < 0.0;
      r = lo ? r - 1.0 : r;
      d = lo ? d + a : d;
      const bool hi = d >= a;
      r = hi ? r + 1.0 : r;
      d = hi ? d - a : d;
    }
    w[i] = d;
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

template <int U, int V, int TM, int TN, int FE, bool PAD, bool LAZY>
__global__ __launch_bounds__(kThreads, 2) void fp64_words_kernel(const Fp64Batch bt) {
  static_assert(FE == 1 || FE == 2 || FE == 4, "reduction period");
  // which product of the batch this workgroup belongs to (uniform, scalar)
  int job = 0;
  while (job + 1 < bt.njobs && (int)blockIdx.x >= bt.tile_start[job + 1]) job++;
  const Fp64Args& a = bt.job[job];
  // split-K: the k-range varies fastest over workgroup ids, so with 8 (or
  // 16, ...) k-ranges each XCD of the round-robin dispatch reads only its
  // own k-range of A and B
  const int bid = (int)blockIdx.x - bt.tile_start[job];
  const int split = a.splits > 1 ? bid % a.splits : 0;
  const int local_bid = a.splits > 1 ? bid / a.splits : bid;
  constexpr int BM = 2 * TM * 16;
  constexpr int BN = 2 * TN * 16;
  constexpr int LDA = kBK + kPadA;
  constexpr int LDB = BN;
  constexpr int NA = BM * kBK / kThreads;  // A slab entries per thread
  constexpr int NB = kBK * BN / kThreads;
  static_assert(NA * kThreads == BM * kBK && NB * kThreads == kBK * BN, "whole slabs per thread");
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

  // Slab elements.  Each stage reads an A slab (BM rows x KR k-terms) and a
  // B slab (KR x BN) with buffer loads: per-stage resources start at
  // (m0, k0) of A and (k0, n0) of B and end at the last entry of the
  // matrix, so rows of A past m and rows of B past k read as zero (the
  // first only feed outputs that are never stored); columns of A past k are
  // zeroed explicitly in the last stage.  Per-thread byte offsets into the
  // slab stay fixed across stages.
  //   whole stages (PAD = false, KR = 16): thread t takes k-term t % 16 of A
  //     rows t / 16 + 16 e, and column t % BN of B k-rows t / BN + (256/BN) e,
  //     so its LDS destinations are affine in e;
  //   padded stages (PAD, KR < 16 real terms in 16 slots): real term kk goes
  //     to slot (kk / L) S + kk % L and the other slots keep their zeros;
  //     elements past the slab are idle: their byte offset lies past every
  //     resource (at most 2^31 - 1 bytes), so they load zero, which they
  //     write to A's pad column (never read) and to B's slot L (a zero slot
  //     when L < S).
  const int KR = a.KR;
  constexpr int AROWS = kThreads / kBK;  // A rows between a thread's elements
  constexpr int BROWS = kThreads / BN;   // B k-rows between a thread's elements
  uint32_t a_off[NA], b_off[NB];
  int a_meta[PAD ? NA : 1], b_meta[PAD ? NB : 1];  // LDS element offset | kk << 16
  int a_dst0 = 0, b_dst0 = 0, t_kk = 0;
  if constexpr (!PAD) {
    const int r0 = tid / kBK, c0 = tid % BN, kb = tid / BN;
    t_kk = tid % kBK;
#pragma unroll
    for (int e = 0; e < NA; e++) a_off[e] = (uint32_t)(((int64_t)(r0 + AROWS * e) * a.lda + t_kk) * 8);
#pragma unroll
    for (int e = 0; e < NB; e++) b_off[e] = (uint32_t)(((int64_t)(kb + BROWS * e) * a.ldb + c0) * 8);
    a_dst0 = r0 * LDA + t_kk;
    b_dst0 = kb * LDB + bswz(kb, c0);  // BROWS is even: every element has kb's parity
  } else {
#pragma unroll
    for (int e = 0; e < NA; e++) {
      const int idx = tid + e * kThreads;
      const bool valid = idx < BM * KR;
      const int r = valid ? idx / KR : 0, kk = valid ? idx % KR : 0;
      const int slot = (kk / a.L) * a.S + kk % a.L;
      a_off[e] = valid ? (uint32_t)(((int64_t)r * a.lda + kk) * 8) : kIdleOffset;
      a_meta[e] = valid ? (r * LDA + slot) | (kk << 16) : kBK | (kBK << 16);
    }
#pragma unroll
    for (int e = 0; e < NB; e++) {
      const int idx = tid + e * kThreads;
      const bool valid = idx < KR * BN;
      const int kk = valid ? idx / BN : 0, c = valid ? idx % BN : 0;
      const int slot = (kk / a.L) * a.S + kk % a.L;
      b_off[e] = valid ? (uint32_t)(((int64_t)kk * a.ldb + c) * 8) : kIdleOffset;
      b_meta[e] = valid ? (slot * LDB + bswz(slot, c)) | (kk << 16) : (a.L * LDB + bswz(a.L, 0)) | (kBK << 16);
    }
  }
  const double p = a.p, q = a.q, bias = a.bias;
  const bool cen = a.centered != 0;
  const bool afix = !cen && a.afix, bfix = !cen && a.bfix;

  double ra[NA], rb[NB];
  auto load_stage = [&](int64_t k0) {
    const int64_t left = a.k - k0;  // real k-terms from k0 on (>= 1)
    const int64_t abytes = ((a.m - m0 - 1) * a.lda + left) * 8;
    const int64_t bbytes = ((left - 1) * a.ldb + (a.n - n0)) * 8;
    const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.A + m0 * a.lda + k0), (short)0, (int)(abytes < 0x7fffffff ? abytes : 0x7fffffff), kBufferWord3);
    const __amdgpu_buffer_rsrc_t br = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(a.B + k0 * a.ldb + n0), (short)0, (int)(bbytes < 0x7fffffff ? bbytes : 0x7fffffff), kBufferWord3);
#pragma unroll
    for (int e = 0; e < NA; e++) ra[e] = buffer_load_f64(ar, a_off[e]);
#pragma unroll
    for (int e = 0; e < NB; e++) rb[e] = buffer_load_f64(br, b_off[e]);
    if constexpr (!PAD) {
      if (left < kBK) {  // the k tail: A's columns past k hold other data
        const bool ok = t_kk < left;
#pragma unroll
        for (int e = 0; e < NA; e++) ra[e] = ok ? ra[e] : 0.0;
      }
    } else if (left < KR) {
      // the k tail: A's terms past k hold other data; B's k-rows past k lie
      // beyond its resource and already read as zero
      const int lim = (int)left;
#pragma unroll
      for (int e = 0; e < NA; e++) ra[e] = (a_meta[e] >> 16) < lim ? ra[e] : 0.0;
    }
  };
  auto store_stage_as = [&](int buf, auto centered) {
    constexpr bool CEN = decltype(centered)::value;
#pragma unroll
    for (int e = 0; e < NA; e++) {
      double w[U];
      split_entry<U, CEN>(ra[e], p, a.alpha, a.ainv, afix, w);
      const int dst = PAD ? (a_meta[PAD ? e : 0] & 0xffff) : a_dst0 + e * AROWS * LDA;
#pragma unroll
      for (int i = 0; i < U; i++) (&As[buf][i][0][0])[dst] = w[i];
    }
#pragma unroll
    for (int e = 0; e < NB; e++) {
      double w[V];
      split_entry<V, CEN>(rb[e], p, a.beta, a.binv, bfix, w);
      const int dst = PAD ? (b_meta[PAD ? e : 0] & 0xffff) : b_dst0 + e * BROWS * LDB;
#pragma unroll
      for (int j = 0; j < V; j++) (&Bs[buf][j][0][0])[dst] = w[j];
    }
  };
  // one uniform branch per stage between the paper's words and centered words
  auto store_stage = [&](int buf) {
    if (cen)
      store_stage_as(buf, std::true_type{});
    else
      store_stage_as(buf, std::false_type{});
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

  const int64_t nstages_all = (a.k + KR - 1) / KR;
  // this split's stages: [s_begin, s_end)
  const int64_t per_split = (nstages_all + a.splits - 1) / a.splits;
  const int64_t s_begin = (int64_t)split * per_split;
  const int64_t s_end = s_begin + per_split < nstages_all ? s_begin + per_split : nstages_all;
  const int lrow = lane & 15, lk = lane >> 4;

  // In-loop reduction (Alg. 1) of one accumulator tile.  The correction-free
  // form leaves values in [-p, 2p) (or the biased range); when the planner
  // could not show that a block started there stays within 2^t (LAZY =
  // false), the two corrections follow.
  auto reduce_one = [&](d4& v) {
#pragma unroll
    for (int r = 0; r < 4; r++) v[r] = fmod_lazy(v[r], p, q, bias);
    if constexpr (!LAZY) {
#pragma unroll
      for (int r = 0; r < 4; r++) {
        double d = v[r];
        d = (d >= p) ? d - p : d;
        v[r] = (d < 0.0) ? d + p : d;
      }
    }
  };
  auto reduce_all = [&]() {
#pragma unroll
    for (int i = 0; i < U; i++)
#pragma unroll
      for (int j = 0; j < V; j++)
#pragma unroll
        for (int x = 0; x < TM; x++)
#pragma unroll
          for (int y = 0; y < TN; y++) reduce_one(acc[i][j][x][y]);
  };

  // Stage s is split into buffer (s - s_begin) & 1 one iteration ahead; its
  // global loads are issued one further iteration ahead, so they are in
  // flight during a whole stage of MFMAs.  One barrier per stage: after it,
  // every wave has finished reading the buffer the next store overwrites.
  int kc = 0;                           // k-steps since the last in-loop reduction
  const int kpb = a.ksteps_per_block;  // FE == 4: k-steps per block (S / 4)
  __syncthreads();  // the zeroed buffers are visible before any store
  if (s_begin < s_end) {
    load_stage(s_begin * KR);
    store_stage(0);
    if (s_begin + 1 < s_end) load_stage((s_begin + 1) * KR);
  }
  lds_barrier();
  // Fragments of one k-step: A's rows for every word and tile row, B's
  // columns for every word and tile column.
  auto read_frags = [&](int buf, int ks, double (&af)[U][TM], double (&bf)[V][TN]) {
#pragma unroll
    for (int i = 0; i < U; i++)
#pragma unroll
      for (int x = 0; x < TM; x++) af[i][x] = As[buf][i][wm + x * 16 + lrow][ks * 4 + lk];
#pragma unroll
    for (int j = 0; j < V; j++)
#pragma unroll
      for (int y = 0; y < TN; y++) bf[j][y] = Bs[buf][j][ks * 4 + lk][bswz(lk, wn + y * 16 + lrow)];
  };
  constexpr int NACC = U * V * TM * TN;
  constexpr int kRedOps = LAZY ? 12 : 32;  // VALU operations of reduce_one (4 values)
  // accumulator t in (i, j, x, y) order
  auto acc_of = [&](int t) -> d4& {
    return acc[t / (V * TM * TN)][(t / (TM * TN)) % V][(t / TN) % TM][t % TN];
  };
  auto mfma_one = [&](int t, const double (&af)[U][TM], const double (&bf)[V][TN]) {
    const int i = t / (V * TM * TN), j = (t / (TM * TN)) % V, x = (t / TN) % TM, y = t % TN;
    acc[i][j][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][x], bf[j][y], acc[i][j][x][y], 0, 0, 0);
  };

  if constexpr (FE < 4) {
    // Blocks of FE k-steps (4 or 8 slots).  The reduction that ends a block
    // is deferred to the start of the next one and interleaved with its
    // first k-step, one accumulator ahead: reduce t + 1, then the MFMA on t.
    // On gfx950 no VALU instruction issues while the SIMD's matrix pipe runs
    // an FP64 MFMA, from the same wave or another, so reductions and MFMAs
    // add up; the interleave keeps either wave of a SIMD ready to issue.
    // The first block of a range reduces its initial value too (harmless:
    // any |x| <= 2^t maps into the restart range); the last block's
    // reduction is left to the epilogue's complete one (its partial sums are
    // within 2^t by the block bound).
    for (int64_t s = s_begin; s < s_end; s++) {
      const int buf = (int)((s - s_begin) & 1);
#pragma unroll
      for (int ks = 0; ks < kBK / 4; ks++) {
        double af[U][TM], bf[V][TN];
        read_frags(buf, ks, af, bf);
        if (ks % FE == 0) {
          reduce_one(acc_of(0));
#pragma unroll
          for (int t = 0; t < NACC; t++) {
            if (t + 1 < NACC) reduce_one(acc_of(t + 1));
            mfma_one(t, af, bf);
          }
        } else {
#pragma unroll
          for (int t = 0; t < NACC; t++) mfma_one(t, af, bf);
        }
        // Nudge the machine schedule toward that order: the fragment reads,
        // then a reduction's VALU operations between MFMAs (left alone, the
        // compiler gathers the MFMAs into bursts; hard scheduling fences
        // enforcing the exact order measured slower).  Only for correction-
        // free blocks of 8 slots (the paper's bound at 45-50 bits and the
        // like), where it measured faster: the grouping costs compile time.
        if constexpr (LAZY && FE == 2) {
        __builtin_amdgcn_sched_group_barrier(0x100, U * TM + V * TN, 0);  // LDS reads
        if (ks % FE == 0) {
          __builtin_amdgcn_sched_group_barrier(0x002, 2 * kRedOps, 0);
#pragma unroll
          for (int t = 0; t + 1 < NACC; t++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, kRedOps, 0);
          }
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        } else {
          __builtin_amdgcn_sched_group_barrier(0x008, NACC, 0);
        }
        }
      }
      if (s + 1 < s_end) {
        store_stage(buf ^ 1);
        if (s + 2 < s_end) load_stage((s + 2) * KR);
      }
      lds_barrier();
    }
  } else {
    for (int64_t s = s_begin; s < s_end; s++) {
      const int buf = (int)((s - s_begin) & 1);
#pragma unroll
      for (int ks = 0; ks < kBK / 4; ks++) {
        double af[U][TM], bf[V][TN];
        read_frags(buf, ks, af, bf);
#pragma unroll
        for (int t = 0; t < NACC; t++) mfma_one(t, af, bf);
        // blocks of any whole number of k-steps, across stages
        if (++kc == kpb) {
          kc = 0;
          reduce_all();
        }
      }
      if (s + 1 < s_end) {
        store_stage(buf ^ 1);
        if (s + 2 < s_end) load_stage((s + 2) * KR);
      }
      lds_barrier();
    }
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
template <int U, int V, int ID, bool WIDE>
struct TileOf {
  static constexpr int tm = fp64_tile_c(ID, U, V, WIDE).tm;
  static constexpr int tn = fp64_tile_c(ID, U, V, WIDE).tn;
};

// Tiles of one product for a given shape.
template <int BM, int BN>
inline int64_t tiles_of(const Fp64Args& a) {
  return ((a.m + BM - 1) / BM) * ((a.n + BN - 1) / BN) * a.splits;
}

template <int U, int V, int ID, int FE, bool PAD, bool LAZY>
int launch_shape(const Fp64Batch& b0, hipStream_t s) {
  constexpr bool WIDE = FE == 4 && !PAD;  // fp64_wide() of the launch's class
  constexpr int TM = TileOf<U, V, ID, WIDE>::tm, TN = TileOf<U, V, ID, WIDE>::tn;
  constexpr int BM = 2 * 16 * TM, BN = 2 * 16 * TN;
  Fp64Batch b = b0;
  int64_t total = 0;
  for (int j = 0; j < b.njobs; j++) {
    // the kernel's 32-bit slab offsets: BM rows of A and 16 k-rows of B
    const Fp64Args& x = b.job[j];
    if (((BM - 1) * x.lda + kBK) * 8 >= ((int64_t)1 << 31) || (kBK * x.ldb + BN) * 8 >= ((int64_t)1 << 31))
      return (int)hipErrorInvalidValue;
    b.tile_start[j] = (int)total;
    total += tiles_of<BM, BN>(b.job[j]);
    if (total > 0x7fffffff) return (int)hipErrorInvalidValue;
  }
  b.tile_start[b.njobs] = (int)total;
  if (total <= 0) return 0;
  TimerTok* t = timer_begin("fp64_words");
  hipExtLaunchKernelGGL((fp64_words_kernel<U, V, TM, TN, FE, PAD, LAZY>), dim3((unsigned)total), dim3(kThreads), 0, s,
                        timer_start(t), timer_stop(t), 0, b);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

}  // namespace fp64w
}  // namespace mmp
