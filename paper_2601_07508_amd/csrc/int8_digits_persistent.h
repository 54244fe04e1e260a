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
  constexpr int IPW = (GROUPS + NW - 1) / NW;   // per wave; the last ones may idle
  __shared__ __attribute__((aligned(1024))) DigitRing<D, BM, BN, 2> sm;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / S::WN) * TM * 16, wn = (wave % S::WN) * TN * 16;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int nbm = (int)((a.m + BM - 1) / BM), nbn = (int)((a.n + BN - 1) / BN);
  const int total = nbm * nbn;
  const int G = (int)gridDim.x;
  // stages per tile: at least one, and within one int32 block (launcher)
  const int nst = (int)(a.kp / kBK8);
  const int64_t planeA = plane_size(a.m, a.kp), planeB = plane_size(a.n, a.kp);
  const int rl = lane >> 2;                                       // row within a 16-row group
  const int ql = (lane & 3) ^ (((lane >> 4) ^ (lane >> 3)) & 3);  // chunk this lane copies

  // Copy offsets of the tile whose stages are being issued: one 1 KB block
  // of a plane per copy, rows past m or n clamped to the last row.  The same
  // copies as digit_tile_loop's, written out again here: routing both
  // through one shared helper changed the code the compiler generates for
  // the main digit GEMM (a longer loop), which this form must not touch.
  uint32_t voff[IPW];  // planes below 4 GB (launcher)
  auto set_offsets = [&](int64_t m0, int64_t n0) {
#pragma unroll
    for (int e = 0; e < IPW; e++) {
      const int t = wv + NW * e;
      if (GROUPS % NW != 0 && t >= GROUPS) {
        voff[e] = 0;  // no copy
      } else if (t < D * BM / 16) {
        const int64_t row = m0 + 16 * (t % (BM / 16)) + rl;
        voff[e] = (uint32_t)plane_at(row < a.m ? row : a.m - 1, 16 * ql, a.kp);
      } else {
        const int64_t row = n0 + 16 * ((t - D * BM / 16) % (BN / 16)) + rl;
        voff[e] = (uint32_t)plane_at(row < a.n ? row : a.n - 1, 16 * ql, a.kp);
      }
    }
  };
  auto issue = [&](int st, int b) {
#pragma unroll
    for (int e = 0; e < IPW; e++) {
      const int t = wv + NW * e;
      if (GROUPS % NW != 0 && t >= GROUPS) continue;  // uniform per wave
      const int8_t* base;
      int plane, row0;
      if (t < D * BM / 16) {
        plane = t / (BM / 16);
        row0 = 16 * (t % (BM / 16));
        base = a.Ad + plane * planeA + (uint32_t)st * 1024u;
      } else {
        const int t2 = t - D * BM / 16;
        plane = t2 / (BN / 16);
        row0 = BM + 16 * (t2 % (BN / 16));
        base = a.Bd + plane * planeB + (uint32_t)st * 1024u;
      }
      __builtin_amdgcn_global_load_lds((const void*)(base + voff[e]),
                                       (__attribute__((address_space(3))) void*)&sm.s[b][plane][row0][0], 16, 0, 0);
    }
  };

  int4v acc[ND][TM][TN];
#pragma unroll
  for (int s = 0; s < ND; s++)
#pragma unroll
    for (int x = 0; x < TM; x++)
#pragma unroll
      for (int y = 0; y < TN; y++) acc[s][x][y] = (int4v){0, 0, 0, 0};
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
  for (;;) {
    const int next = item + G;
    for (int st = 0; st < nst; st++) {
      // this wave's copies of stage st are complete; the barrier extends
      // that to every wave and ends the reads of the previous stage, whose
      // buffer the next copies overwrite
      wait_vm<0>();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      // one issue site: the tile's next stage, or the next tile's first
      int st_n = st + 1;
      if (st_n == nst) {
        st_n = next < total ? 0 : -1;
        if (st_n == 0) {
          int ti, tj;
          tile_coords(next, total, nbm, nbn, ti, tj);
          set_offsets((int64_t)ti * BM, (int64_t)tj * BN);
        }
      }
      if (st_n >= 0) issue(st_n, b ^ 1);
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
      b ^= 1;
    }
    // fold the tile's digit-weight sums into C and clear them; 16x16x64
    // INT8 MFMA output layout: value (i & 3) of lane j + 16 (i >> 2)
#pragma unroll
    for (int x = 0; x < TM; x++)
#pragma unroll
      for (int y = 0; y < TN; y++) {
        const int64_t col = (int64_t)tni * BN + wn + y * 16 + lrow;
#pragma unroll
        for (int r = 0; r < 4; r++) {
          int w[ND];
#pragma unroll
          for (int s = 0; s < ND; s++) w[s] = acc[s][x][y][r];
          double t;
          if constexpr (D >= 3)
            t = fold_short<ND>(w, p, q);
          else
            t = fold_weights<ND>(w, p, q);
          const int64_t row = (int64_t)tmi * BM + wm + x * 16 + (lane >> 4) * 4 + r;
          if (row < a.m && col < a.n) a.C[row * a.ldc + col] = t + 0.0;
        }
      }
#pragma unroll
    for (int s = 0; s < ND; s++)
#pragma unroll
      for (int x = 0; x < TM; x++)
#pragma unroll
        for (int y = 0; y < TN; y++) acc[s][x][y] = (int4v){0, 0, 0, 0};
    if (next >= total) break;  // uniform; nothing was issued past this tile
    item = next;
    tile_coords(item, total, nbm, nbn, tmi, tni);
  }
}

}  // namespace i8d
}  // namespace mmp
