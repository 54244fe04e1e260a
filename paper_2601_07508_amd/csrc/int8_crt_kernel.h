// Multi-modular product (Section 5.2's setting): one integer pair A, B
// against many moduli.  The digit products of the integers are formed once
// (k within one int32 block, digit loop of int8_digits_kernel.h) and every
// modulus reduces the same digit-weight sums in the epilogue:
//     C_i = sum_s 256^s D_s mod p_i.
//
// The weights do not depend on the modulus, so the epilogue first combines
// them, once per output, into exact groups of three,
//     G_j = D_3j + 256 D_3j+1 + 65536 D_3j+2,
// |G_j| <= (2^31 - 1) 65793 < 2^47.01 (an integer, exact in binary64), and
// each modulus then runs Horner's rule over the groups with the scale 2^24:
// ceil((2D - 1) / 3) - 1 steps instead of 2D - 2, over the groups as they
// are when every modulus of the launch is large next to them (fold_direct;
// the launcher checks Gmax <= (2^27 - 2) p), else over the groups each
// reduced first (fold_groups).
#pragma once
#include <type_traits>
#include "int8_fold.h"

namespace mmp {
namespace i8d {

constexpr int kMaxPrimes = 64;
struct CrtArgs {
  const int8_t* Ad;  // D planes of m x kp (16-row blocks, plane_at)
  const int8_t* Bd;  // D planes of n x kp
  int64_t m, n, kp, ldc;
  int nprimes;
  int direct;  // every modulus allows fold_direct for these groups
  double p[kMaxPrimes];
  double q[kMaxPrimes];
  double* C[kMaxPrimes];
};

template <int D>
__global__ __launch_bounds__(I8Shape<D>::THREADS, I8Shape<D>::GROUPS_PER_CU) void crt_gemm_kernel(
    const CrtArgs a) {
  using S = I8Shape<D>;
  constexpr int ND = 2 * D - 1;
  constexpr int NG = (ND + 2) / 3;
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  __shared__ __attribute__((aligned(1024))) DigitRing<D, BM, BN, S::STAGES> sm;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int nbm = (int)((a.m + BM - 1) / BM), nbn = (int)((a.n + BN - 1) / BN);
  int tmi, tni;
  tile_coords(blockIdx.x, nbm * nbn, nbm, nbn, tmi, tni);
  const int64_t m0 = (int64_t)tmi * BM, n0 = (int64_t)tni * BN;

  int4v acc[ND][TM][TN];
#pragma unroll
  for (int s = 0; s < ND; s++)
#pragma unroll
    for (int x = 0; x < TM; x++)
#pragma unroll
      for (int y = 0; y < TN; y++) acc[s][x][y] = (int4v){0, 0, 0, 0};
  // one int32 block covers the whole k (checked by the launcher)
  digit_tile_loop<D, S>(a.Ad, a.Bd, a.m, a.n, a.kp, m0, n0, 0, a.kp / kBK8, a.kp / kBK8 + 1, sm, acc, [] {});

  // the weights in exact groups of three, shared by every modulus
  double g[TM][TN][4][NG];
#pragma unroll
  for (int x = 0; x < TM; x++)
#pragma unroll
    for (int y = 0; y < TN; y++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        int w[ND];
#pragma unroll
        for (int s = 0; s < ND; s++) w[s] = acc[s][x][y][r];
#pragma unroll
        for (int j = 0; j < NG; j++) g[x][y][r][j] = weight_group<ND>(w, j);
      }

  // One pass over the moduli per fold form (a uniform choice).  Each
  // modulus's C is written once and not read here again: streaming
  // (nontemporal) stores keep the 32 outputs from displacing the digit
  // planes other tiles read from L2.  A whole tile inside C (uniform) takes
  // no per-element bounds and one row pointer per output row.
  const int lrow = lane & 15;
  const int64_t row0 = m0 + wm + (lane >> 4) * 4, col0 = n0 + wn + lrow;
  const bool whole = m0 + BM <= a.m && n0 + BN <= a.n;
  auto moduli = [&](auto directc) {
    constexpr bool DIRECT = decltype(directc)::value;
    for (int pi = 0; pi < a.nprimes; pi++) {
      const double p = a.p[pi], q = a.q[pi];
      double* const C = a.C[pi];
      auto fold = [&](int x, int y, int r) {
        // fold_direct over weight groups never returns -0 (an int converted
        // to binary64, or an exact fma or sum that is zero, is +0 unless
        // both terms are -0); the other form's result is normalised
        if constexpr (DIRECT)
          return fold_direct<NG>(g[x][y][r], p, q);
        else
          return fold_groups<NG>(g[x][y][r], p, q) + 0.0;
      };
      if (whole) {
        double* const c0 = C + row0 * a.ldc + col0;
#pragma unroll
        for (int x = 0; x < TM; x++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            double* const cr = c0 + (int64_t)(x * 16 + r) * a.ldc;
#pragma unroll
            for (int y = 0; y < TN; y++) __builtin_nontemporal_store(fold(x, y, r), &cr[y * 16]);
          }
      } else {
#pragma unroll
        for (int x = 0; x < TM; x++)
#pragma unroll
          for (int y = 0; y < TN; y++) {
            const int64_t col = col0 + y * 16;
#pragma unroll
            for (int r = 0; r < 4; r++) {
              const double t = fold(x, y, r);
              const int64_t row = row0 + x * 16 + r;
              if (row < a.m && col < a.n) __builtin_nontemporal_store(t, &C[row * a.ldc + col]);
            }
          }
      }
    }
  };
  if (a.direct)
    moduli(std::true_type{});
  else
    moduli(std::false_type{});
}

}  // namespace i8d
}  // namespace mmp
