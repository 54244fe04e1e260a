// Folds of digit-weight sums in groups of three (the INT8-digit form's
// int32 accumulators D_s, value sum_s 256^s D_s): the multi-modular
// epilogue's (int8_crt_kernel.h) and the short-tile fold of the persistent
// digit GEMM (int8_digits_persistent.h).  All steps are Section 2.1's
// binary64 arithmetic with exact results; each bound is stated where used.
#pragma once
#include "int8_digits_kernel.h"

namespace mmp {
namespace i8d {

// G_j = D_3j + 256 D_3j+1 + 65536 D_3j+2 (missing terms zero), exact for
// |D_s| < 2^31: |G_j| < 2^31 65793 < 2^47.01.
template <int ND>
__device__ __forceinline__ double weight_group(const int (&w)[ND], int j) {
  double v = (double)w[3 * j];
  if (3 * j + 1 < ND) v = fma(256.0, (double)w[3 * j + 1], v);
  if (3 * j + 2 < ND) v = fma(65536.0, (double)w[3 * j + 2], v);
  return v;
}

// Alg. 1 with the quotient rounded to nearest and no corrections: for an
// integer x with |x| < 2^53, c = floor(fl(x q + 1/2)) and d = x - c p
// (exact in one fma when |d| < 2^53).  With q = fl(1/p), fl(x q + 1/2) is
// within |x / p| 2^-52 + 2^-54 of x / p + 1/2, so |d| <= p/2 + |x| 2^-52 +
// p 2^-54.
__device__ __forceinline__ double reduce_near(double x, double p, double q) {
  return fma(-floor(fma(x, q, 0.5)), p, x);
}

// sum_j 2^24j g[j] mod p in [0, p) for integers |g[j]| < 2^47.01, p < 2^52:
//   t = reduce_near(g[NG-1]); t = reduce_near(2^24 t) + reduce_near(g[j]),
// j = NG-2 .. 0; one complete reduction ends it.  Each reduced group lies
// within p/2 + 1 of zero (|g| 2^-52 < 2^-4.9).  If |t| <= T, then 2^24 t is
// exact (a power of two), its reduction lies within p/2 + 2^-28 T + p 2^-54
// of zero, and the new t within p + 2 + 2^-28 T: T = p (1 + 2^-27) + 2
// holds at every step, below 2^53, so every step is exact.  The final
// quotient floor(t q) is then within one of t / p, which one correction on
// each side absorbs.
template <int NG>
__device__ __forceinline__ double fold_groups(const double (&g)[NG], double p, double q) {
  double t = reduce_near(g[NG - 1], p, q);
#pragma unroll
  for (int j = NG - 2; j >= 0; j--) t = reduce_near(16777216.0 * t, p, q) + reduce_near(g[j], p, q);
  return fmod_full(t, p, q);
}

// sum_j 2^24j g[j] mod p in [0, p) when the groups are small next to p:
// |g[j]| <= Gmax with Gmax <= (2^27 - 2) p (and Gmax < 2^47.01, p < 2^52).
// Horner's rule then runs over the groups directly, t = reduce_near(2^24 t)
// + g[j] from t = g[NG-1], with no reduction of the groups themselves.  If
// |t| <= p + Gmax, the quotient argument |2^24 t / p| <= 2^24 (1 + Gmax / p)
// < 2^51, so its error is below 1/2, the reduction lies within p of zero
// and the new |t| <= p + Gmax again (below 2^53): every step is exact.  It
// ends with one more rounded reduction: |t / p| <= 2^27, so the quotient's
// error is below 2^-24 and d = reduce_near(t) lies within p/2 + 1 of zero;
// adding p to a negative d gives the residue in [0, p) (three operations
// fewer than Alg. 1 with both corrections).  For digit-weight sums over K
// k-terms of D-digit operands, Gmax = 65793 K D 2^14 (direct_fold_ok).
template <int NG>
__device__ __forceinline__ double fold_direct(const double (&g)[NG], double p, double q) {
  double t = g[NG - 1];
#pragma unroll
  for (int j = NG - 2; j >= 0; j--) t = reduce_near(16777216.0 * t, p, q) + g[j];
  const double d = reduce_near(t, p, q);
  return d < 0.0 ? d + p : d;
}

// The persistent digit GEMM's tiles: whole k at most 1024 terms, D <= 7 and
// p >= 2^16 (three or more digits), so Gmax = 65793 * 1024 * 7 * 2^14 <
// 2^42.82 <= 2^26.82 p: fold_direct over the groups of w.
template <int ND>
__device__ __forceinline__ double fold_short(const int (&w)[ND], double p, double q) {
  constexpr int NG = (ND + 2) / 3;
  double g[NG];
#pragma unroll
  for (int j = 0; j < NG; j++) g[j] = weight_group<ND>(w, j);
  return fold_direct<NG>(g, p, q);
}

}  // namespace i8d
}  // namespace mmp
