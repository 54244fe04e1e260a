// Persistent form of the digit GEMM (int8_digits_kernel.h) for one product
// with many output tiles of few k-stages each, such as m = n = 16384 with
// k = 256 (four stages a tile).  There a workgroup per tile spends most of
// its life waiting: each of its stages is a full copy latency behind the
// previous one, and a new workgroup starts with an empty ring.  Here one
// workgroup per resident slot walks the tiles w, w + G, w + 2G, ... (G
// workgroups; with G a multiple of 8 every tile stays on the XCD the
// one-tile-per-workgroup launch puts it on) and its two-stage copy ring runs
// across tile boundaries: the next tile's first stage is in flight while the
// current tile's last stage is multiplied, folded and stored.  The digit
// products, fold and output are those of int8_digits_gemm_kernel, whole k
// per tile (no split-K) within one exact int32 block, so each tile folds
// once, at its end, straight into C; from three digits on (p >= 2^16) with
// fold_short, which the tiles' short k (at most 1024 terms) allows.
#pragma once
#include <type_traits>

#include "int8_fold.h"

namespace mmp {
namespace i8d {

template <int D>
__global__ __launch_bounds__((I8Shape<D>::THREADS), (I8Shape<D>::GROUPS_PER_CU)) void
int8_digits_gemm_persistent_kernel(const GemmArgs a) {
  using S = I8Shape<D>;
  static_assert(S::STAGES == 2, "two-stage ring");
  constexpr int ND = 2 * D - 1;
  constexpr int BM = S::BM, BN = S::BN, TM = S::TM, TN = S::TN;
  constexpr int NW = S::WM * S::WN;
  constexpr int GROUPS = D * (BM + BN) / 16;  // 1 KB copy instructions per stage
  constexpr int IPW = GROUPS / NW;             // per wave
  // the first half of the waves copies A's blocks, the second half B's
  static_assert(GROUPS % NW == 0 && D * BM / 16 == (NW / 2) * IPW && D * BN / 16 == (NW / 2) * IPW,
                "copies split evenly between A's and B's waves");
  __shared__ __attribute__((aligned(1024))) DigitRing<D, BM, BN, 2> sm;
  constexpr uint32_t STAGE_BYTES = sizeof(sm.s[0]);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const bool copies_a = wv < NW / 2;
  const int nbm = (int)((a.m + BM - 1) / BM), nbn = (int)((a.n + BN - 1) / BN);
  const int total = nbm * nbn;
  const int G = (int)gridDim.x;
  // stages per tile: at least one, and within one int32 block (launcher)
  const int nst = (int)(a.kp / kBK8);
  const int rl = lane >> 2;                                       // row within a 16-row group
  const int ql = (lane & 3) ^ (((lane >> 4) ^ (lane >> 3)) & 3);  // chunk this lane copies

  // This wave's copies: block c = (wave mod NW/2) IPW + e of its operand,
  // digit plane c / (rows / 16), 16-row part c mod (rows / 16).  Each copy
  // moves one 1 KB block of a plane; the lane offsets (voff, from the
  // operand's first plane: all its planes lie below 4 GB, launcher) hold
  // the plane and the tile's rows, rows past m or n clamped to the last
  // row, so a stage's copies add only the stage's 1 KB step.  The same
  // copies as digit_tile_loop's, written out again here: routing both
  // through one shared helper changed the code the compiler generates for
  // the main digit GEMM (a longer loop), which this form must not touch.
  const int8_t* const opbase = copies_a ? a.Ad : a.Bd;
  const int64_t oprows = copies_a ? a.m : a.n;
  const int64_t opplane = plane_size(oprows, a.kp);
  constexpr int PARTS = BM / 16;  // == BN / 16
  static_assert(BM == BN, "square tiles: one part count for both operands");
  const int c0 = (copies_a ? wv : wv - NW / 2) * IPW;
  uint32_t lds_off[IPW];  // each copy's row block in stage 0 of the ring
#pragma unroll
  for (int e = 0; e < IPW; e++) {
    const int c = c0 + e, plane = c / PARTS, part = c % PARTS;
    lds_off[e] = (uint32_t)((plane * (BM + BN) + (copies_a ? 0 : BM) + 16 * part) * 64);
  }
  uint32_t voff[IPW];
  auto set_offsets = [&](int64_t m0, int64_t n0) {
    const int64_t r0 = copies_a ? m0 : n0;
#pragma unroll
    for (int e = 0; e < IPW; e++) {
      const int c = c0 + e, plane = c / PARTS, part = c % PARTS;
      const int64_t row = r0 + 16 * part + rl;
      voff[e] = (uint32_t)(plane * opplane + plane_at(row < oprows ? row : oprows - 1, 16 * ql, a.kp));
    }
  };
  auto issue = [&](int st, int b) {
    const int8_t* const base = opbase + (uint32_t)st * 1024u;
    const uint32_t ring = (uint32_t)b * STAGE_BYTES;
#pragma unroll
    for (int e = 0; e < IPW; e++)
      __builtin_amdgcn_global_load_lds(
          (const void*)(base + voff[e]),
          (__attribute__((address_space(3))) void*)((__attribute__((address_space(3))) int8_t*)&sm.s[0][0][0][0] +
                                                    ring + lds_off[e]),
          16, 0, 0);
  };

  int4v acc[ND][TM][TN];  // each tile's first stage sets them
  const double p = a.p, q = a.q;

  // one tile per outer iteration; the last stage of a tile issues the first
  // copies of the next tile of this workgroup (item + G)
  int item = (int)blockIdx.x;
  if (item >= total) return;  // uniform: the launcher sizes G <= total
  int tmi, tni;
  tile_coords(item, total, nbm, nbn, tmi, tni);
  set_offsets((int64_t)tmi * BM, (int64_t)tni * BN);
  issue(0, 0);
  int b = 0;
  const int lrow = lane & 15, lq = lane >> 4;
  // Store instructions the whole-tile epilogue issues (one per output
  // element: a lane's elements are never adjacent, so none merge).  Vector
  // memory instructions complete in issue order for the vmcnt counter, so
  // after that epilogue the next tile's first stage, whose copies were
  // issued before those stores, waits only until that many remain.
  constexpr int NSTORES = TM * TN * 4;
  bool stores_behind = false;
  int nti = 0, ntj = 0;  // the next tile's coordinates
  for (;;) {
    const int next = item + G;
    for (int st = 0; st < nst; st++) {
      // this wave's copies of stage st are complete; the barrier extends
      // that to every wave and ends the reads of the previous stage, whose
      // buffer the next copies overwrite
      if (st == 0 && stores_behind)
        wait_vm<NSTORES>();
      else
        wait_vm<0>();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      // one issue site: the tile's next stage, or the next tile's first
      // (whose copy offsets the previous stage set, or this one if it is
      // the tile's only stage)
      int st_n = st + 1;
      if (st_n == nst) {
        st_n = next < total ? 0 : -1;
        if (nst == 1 && st_n == 0) {
          tile_coords(next, total, nbm, nbn, nti, ntj);
          set_offsets((int64_t)nti * BM, (int64_t)ntj * BN);
        }
      }
      if (st_n >= 0) issue(st_n, b ^ 1);
      int4v bf[D][TN], af[D][TM];
#pragma unroll
      for (int j = 0; j < D; j++)
#pragma unroll
        for (int y = 0; y < TN; y++) {
          const int r = BM + wn + y * 16 + lrow;
          bf[j][y] = *(const int4v*)(&sm.s[b][j][r][swz(r, lq)]);
        }
#pragma unroll
      for (int i = 0; i < D; i++)
#pragma unroll
        for (int x = 0; x < TM; x++) {
          const int r = wm + x * 16 + lrow;
          af[i][x] = *(const int4v*)(&sm.s[b][i][r][swz(r, lq)]);
        }
      // A tile's first stage starts every digit weight from zero: the first
      // product of each weight (i = max(0, s - D + 1)) takes a zero
      // accumulator operand, so no instruction clears the accumulators
      // between tiles.
      auto mma = [&](auto firstc) {
        constexpr bool FIRST = decltype(firstc)::value;
#pragma unroll
        for (int i = 0; i < D; i++) {
#pragma unroll
          for (int j = 0; j < D; j++)
#pragma unroll
            for (int x = 0; x < TM; x++)
#pragma unroll
              for (int y = 0; y < TN; y++) {
                const bool fresh = FIRST && i == (i + j > D - 1 ? i + j - (D - 1) : 0);
                acc[i + j][x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                    af[i][x], bf[j][y], fresh ? (int4v){0, 0, 0, 0} : acc[i + j][x][y], 0, 0, 0);
              }
        }
      };
      // Up to three digits the products run at raised wave priority: the
      // SIMD's other waves fold, store and wait for copies in between, and
      // with these short bursts (36 MFMAs a stage) the matrix pipe stays
      // fuller when a burst issues first (measured: 1-2% at 16384^2 x 256;
      // at five digits the same was 5% slower, at four and seven neutral)
      if constexpr (D <= 3) __builtin_amdgcn_s_setprio(1);
      if (st == 0)
        mma(std::true_type{});
      else
        mma(std::false_type{});
      if constexpr (D <= 3) __builtin_amdgcn_s_setprio(0);
      // the next tile's copy offsets, once this tile's last copies are
      // issued, behind this stage's products
      if (st == nst - 2 && next < total) {
        tile_coords(next, total, nbm, nbn, nti, ntj);
        set_offsets((int64_t)nti * BM, (int64_t)ntj * BN);
      }
      b ^= 1;
    }
    // fold the tile's digit-weight sums into C; 16x16x64 INT8 MFMA output
    // layout: value (i & 3) of lane j + 16 (i >> 2).  C is written once and
    // not read here again: streaming (nontemporal) stores keep it from
    // displacing the digit planes the next tiles read from L2.
    auto fold_at = [&](int x, int y, int r) {
      int w[ND];
#pragma unroll
      for (int s = 0; s < ND; s++) w[s] = acc[s][x][y][r];
      if constexpr (D >= 3)
        return fold_short<ND>(w, p, q);
      else
        return fold_weights<ND>(w, p, q);
    };
    const int64_t row0 = (int64_t)tmi * BM + wm + (lane >> 4) * 4, col0 = (int64_t)tni * BN + wn + lrow;
    stores_behind = (int64_t)(tmi + 1) * BM <= a.m && (int64_t)(tni + 1) * BN <= a.n;
    if (stores_behind) {
      // whole tile inside C (uniform): no per-element bounds, one row
      // pointer per output row and the column steps as immediate offsets
      double* const c0 = a.C + row0 * a.ldc + col0;
#pragma unroll
      for (int x = 0; x < TM; x++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          double* const cr = c0 + (int64_t)(x * 16 + r) * a.ldc;
#pragma unroll
          for (int y = 0; y < TN; y++) {
            // fold_short never returns -0: (double) of an int and an exact
            // fma or sum that is zero give +0 unless both terms are -0
            if constexpr (D >= 3)
              __builtin_nontemporal_store(fold_at(x, y, r), &cr[y * 16]);
            else
              __builtin_nontemporal_store(fold_at(x, y, r) + 0.0, &cr[y * 16]);
          }
        }
    } else {
#pragma unroll
      for (int x = 0; x < TM; x++)
#pragma unroll
        for (int y = 0; y < TN; y++) {
          const int64_t col = col0 + y * 16;
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int64_t row = row0 + x * 16 + r;
            const double t = fold_at(x, y, r);
            if (row < a.m && col < a.n) __builtin_nontemporal_store(t + 0.0, &a.C[row * a.ldc + col]);
          }
        }
    }
    if (next >= total) break;  // uniform; nothing was issued past this tile
    item = next;
    tmi = nti;
    tni = ntj;
  }
}

}  // namespace i8d
}  // namespace mmp
