// One launch for the digit planes and one for the digit GEMM of a whole batch
// of INT8-form products, whatever their digit counts (the batched block
// products the paper's closing perspective suggests, Section 6).
//
// The job table travels in the kernel arguments (up to kMaxMixedJobs
// products), so a captured graph replays it as it was.
//   - digitize_batch_kernel: the workgroups of every product's row part (A)
//     and column part (B) one after another; each workgroup finds its product
//     and runs that product's digit count's code (a uniform branch).
//   - int8_batch_gemm_kernel: a persistent grid over the (product, output
//     tile) work items of all products; a workgroup strides over the items
//     and runs each with its product's digit count.  Every digit count uses
//     4 waves (64 x 64 tiles up to 4 digits, 64 x 32 beyond), so one launch
//     shape serves all; the LDS ring is sized for the largest digit count of
//     the launch.
#pragma once
#include <hip/hip_runtime.h>

#include "int8_digitize_kernel.h"
#include "int8_digits_kernel.h"

namespace mmp {
namespace i8d {

constexpr int kMaxMixedJobs = 64;

struct MixedJob {
  const double* A;  // entries in [0, p), row-major
  const double* B;
  int8_t* Ad;  // D planes of m x kp
  int8_t* Bd;  // D planes of n x kp
  double* C;
  int64_t m, n, k, lda, ldb, ldc, kp;
  double p, q;
  int64_t top;               // 127 (256^D - 1) / 255
  int64_t stages_per_block;  // LDS stages between folds
  int D;
  int vec;          // A's rows start 16-byte aligned (aligned base, even lda)
  int dig_start;    // first digitize workgroup of this product (row part, then column part)
  int dig_cols;     // first column-part workgroup
  int gx, gy;       // row part: 128-column chunks x 16-row groups (strided)
  int tile_start;   // first GEMM work item of this product
};

struct MixedBatch {
  int njobs;
  int dig_total;   // digitize workgroups
  int tile_total;  // GEMM work items
  MixedJob job[kMaxMixedJobs];
};

// the product that work item w belongs to, given ascending starts
template <class F>
__device__ __forceinline__ int find_job(const MixedBatch& b, int w, F start) {
  int lo = 0, hi = b.njobs - 1;
  while (lo < hi) {  // uniform: w is the same in every lane
    const int mid = (lo + hi + 1) / 2;
    if (start(b.job[mid]) <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int D>
__device__ __forceinline__ void digitize_item(const MixedJob& a, int local, uint8_t* lds) {
  const ResidueIn in{a.A, (int64_t)a.p, a.top};
  const int rows_items = a.dig_cols - a.dig_start;
  if (local < rows_items) {
    const ResidueIn ia = in;
    if (a.vec)
      digitize_rows_part<D, ResidueIn, true>(ia, a.m, a.k, a.lda, a.kp, a.Ad, local % a.gx, local / a.gx, a.gy);
    else
      digitize_rows_part<D, ResidueIn, false>(ia, a.m, a.k, a.lda, a.kp, a.Ad, local % a.gx, local / a.gx, a.gy);
  } else {
    const ResidueIn ib{a.B, (int64_t)a.p, a.top};
    digitize_cols_part<D, ResidueIn>(ib, a.k, a.n, a.ldb, a.kp, a.Bd, local - rows_items,
                                     *reinterpret_cast<uint8_t(*)[D][64][64 + 4]>(lds));
  }
}

__global__ __launch_bounds__(256) void digitize_batch_kernel(const MixedBatch b) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[kMaxDigits * 64 * (64 + 4)];
  const int w = (int)blockIdx.x;
  const int j = find_job(b, w, [](const MixedJob& x) { return x.dig_start; });
  const MixedJob& a = b.job[j];
  const int local = w - a.dig_start;
  switch (a.D) {
    case 1: digitize_item<1>(a, local, lds); break;
    case 2: digitize_item<2>(a, local, lds); break;
    case 3: digitize_item<3>(a, local, lds); break;
    case 4: digitize_item<4>(a, local, lds); break;
    case 5: digitize_item<5>(a, local, lds); break;
    case 6: digitize_item<6>(a, local, lds); break;
    default: digitize_item<7>(a, local, lds); break;
  }
}

// 4 waves for every digit count: 64 x 64 tiles of 32 x 32 wave tiles up to
// 4 digits (the digit GEMM's own shape there), 64 x 32 tiles of 16 x 32 wave
// tiles beyond (with every digit count's code in one kernel, the 5-digit
// 32 x 32 accumulators spill); two-stage ring.
template <int D>
struct MixedShape {
  static constexpr bool WIDE = D <= 4;
  static constexpr int WM = WIDE ? 2 : 4, WN = WIDE ? 2 : 1, TM = WIDE ? 2 : 1, TN = 2;
  static constexpr int BM = 64, BN = WIDE ? 64 : 32;
  static constexpr int THREADS = 256;
  static constexpr int STAGES = 2;
};

constexpr int64_t mixed_ring_bytes(int D) { return (int64_t)2 * D * (64 + (D <= 4 ? 64 : 32)) * 64; }
constexpr int mixed_bn(int D) { return D <= 4 ? 64 : 32; }

// One output tile of product a: the digit loop over its whole k, folds into
// binary64 residues, one store.
template <int D>
__device__ __forceinline__ void gemm_item(const MixedJob& a, int local, int8_t* lds) {
  using S = MixedShape<D>;
  constexpr int ND = 2 * D - 1;
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  auto& sm = *reinterpret_cast<DigitRing<D, BM, BN, S::STAGES>*>(lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int nbm = (int)((a.m + BM - 1) / BM), nbn = (int)((a.n + BN - 1) / BN);
  int tmi, tni;
  tile_coords(local, nbm * nbn, nbm, nbn, tmi, tni);
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
  digit_tile_loop<D, S>(a.Ad, a.Bd, a.m, a.n, a.kp, m0, n0, 0, a.kp / kBK8, a.stages_per_block, sm, acc, fold);
  // 16x16x64 INT8 MFMA output layout: value (i & 3) of lane j + 16 (i >> 2)
  const int lrow = lane & 15;
#pragma unroll
  for (int x = 0; x < TM; x++)
#pragma unroll
    for (int y = 0; y < TN; y++) {
      const int64_t col = n0 + wn + y * 16 + lrow;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t row = m0 + wm + x * 16 + (lane >> 4) * 4 + r;
        if (row < a.m && col < a.n) __builtin_nontemporal_store(F[x][y][r] + 0.0, &a.C[row * a.ldc + col]);
      }
    }
}

__global__ __launch_bounds__(256, 2) void int8_batch_gemm_kernel(const MixedBatch b) {
  extern __shared__ __attribute__((aligned(1024))) int8_t lds[];
  for (int w = (int)blockIdx.x; w < b.tile_total; w += (int)gridDim.x) {
    const int j = find_job(b, w, [](const MixedJob& x) { return x.tile_start; });
    const MixedJob& a = b.job[j];
    const int local = w - a.tile_start;
    __syncthreads();  // every wave is done with the previous item's ring
    switch (a.D) {
      case 1: gemm_item<1>(a, local, lds); break;
      case 2: gemm_item<2>(a, local, lds); break;
      case 3: gemm_item<3>(a, local, lds); break;
      case 4: gemm_item<4>(a, local, lds); break;
      case 5: gemm_item<5>(a, local, lds); break;
      case 6: gemm_item<6>(a, local, lds); break;
      default: gemm_item<7>(a, local, lds); break;
    }
  }
}

}  // namespace i8d
}  // namespace mmp
