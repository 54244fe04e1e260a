// Planner: word counts, scaling parameters, block size and tile for one
// product.  Pure host integer arithmetic; touches no device.
//
// Paper passages implemented here:
//   alpha = ceil(p^(1/u))                       Section 3.1, Alg. 4
//   block size, (1,1): eq. lambda-sw            Section 2.2
//   block size, (u,v): lambda alpha beta + p - 1 <= 2^t, eq. cAcB, Prop. UVMW
//   (u,v) choice by bitsize and cost            Section 3.3, Table tab.summary
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "mmp_internal.h"

namespace mmp {

typedef unsigned __int128 u128;

uint64_t iroot_ceil(uint64_t p, int u) {
  if (u <= 1) return p;
  // start from the floating-point root, then fix up with exact powers
  uint64_t a = (uint64_t)std::llround(std::pow((double)p, 1.0 / u));
  if (a < 1) a = 1;
  auto pow_ge = [&](uint64_t base) {  // base^u >= p, exact
    u128 r = 1;
    for (int i = 0; i < u; i++) {
      r *= base;
      if (r >= p) return true;
    }
    return r >= p;
  };
  while (!pow_ge(a)) a++;
  while (a > 1 && pow_ge(a - 1)) a--;
  return a;
}

bool supported_words(int u, int v) {
  return u >= 1 && v >= 1 && u <= kMaxWords && v <= kMaxWords && u * v <= kMaxWordProducts;
}

// Largest word product the paper's bound charges per k-term.
static u128 word_product_bound(uint64_t p, int u, int v) {
  if (u == 1 && v == 1) return (u128)(p - 1) * (u128)(p - 1);  // eq. lambda-sw
  return (u128)iroot_ceil(p, u) * (u128)iroot_ceil(p, v);     // eq. cAcB
}

int64_t paper_lambda(uint64_t p, int u, int v) {
  if (p < 5 || p >= kPMax) return 0;
  u128 w = word_product_bound(p, u, v);
  u128 room = (u128)kTwoT - p + 1;  // lambda w + p - 1 <= 2^t
  u128 lam = room / w;
  if (lam > (u128)INT64_MAX) lam = INT64_MAX;
  return (int64_t)lam;
}

bool extended_block_ok(uint64_t p, int u, int v, int64_t L) {
  // The biased reduction leaves [-2^t, -2^t + 4p); L non-negative terms of
  // at most w keep every partial sum within [-2^t, 2^t] if
  // L w + 4p - 1 <= 2^(t+1).
  u128 w = word_product_bound(p, u, v);
  return (u128)L * w + 4 * (u128)p - 1 <= 2 * (u128)kTwoT;
}

int64_t extended_lambda(uint64_t p, int u, int v) {
  if (p < 5 || p >= kPMax) return 0;
  u128 w = word_product_bound(p, u, v);
  u128 room = 2 * (u128)kTwoT - 4 * (u128)p + 1;
  u128 lam = room / w;
  if (lam > (u128)INT64_MAX) lam = INT64_MAX;
  return (int64_t)lam;
}

// Centered words (a variant of Alg. 4 derived for this library).  An entry
// x in [0, p) becomes x~ = x - p when 2x > p, so |x~| <= h = floor(p / 2),
// and is split as x~ = sum_i alpha^i w_i with quotients rounded to nearest:
// r = floor(fl(t fl(1/alpha) + 1/2)), w = t - r alpha.  The estimate is
// within |t / alpha| 2^-52 of t / alpha, so |w| <= alpha / 2 + |t| 2^-52 <
// alpha / 2 + 1 for every word but the last (|t| < 2^51), and the last, the
// final quotient, is at most h / alpha^(u-1) + 2.
uint64_t centered_word_bound(uint64_t p, int u) {
  const uint64_t h = p / 2;
  if (u <= 1) return h;
  const uint64_t a = iroot_ceil(p, u);
  u128 apow = 1;
  for (int i = 0; i < u - 1; i++) apow *= a;
  const uint64_t top = (uint64_t)((u128)h / apow) + 2;
  const uint64_t low = a / 2 + 1;
  return top > low ? top : low;
}

// The centered in-loop reduction c = floor(fl(x q + 1/2)), d = x - c p maps
// any |x| <= 2^t to |d| <= p/2 + 2.25 (the quotient estimate is within
// 2/p + 2^-54 of x/p + 1/2); R = floor(p/2) + 4 bounds it with margin.  A
// block of L terms, each of magnitude at most W = bound(u) bound(v), keeps
// every partial sum within [-2^t, 2^t] if R + L W <= 2^t.
static u128 centered_start(uint64_t p) { return (u128)(p / 2) + 4; }

bool centered_block_ok(uint64_t p, int u, int v, int64_t L) {
  const u128 w = (u128)centered_word_bound(p, u) * (u128)centered_word_bound(p, v);
  return centered_start(p) + (u128)L * w <= (u128)kTwoT;
}

int64_t centered_lambda(uint64_t p, int u, int v) {
  if (p < 5 || p >= kPMax) return 0;
  const u128 w = (u128)centered_word_bound(p, u) * (u128)centered_word_bound(p, v);
  const u128 start = centered_start(p);
  if (start >= (u128)kTwoT || w == 0) return 0;
  u128 lam = ((u128)kTwoT - start) / w;
  if (lam > (u128)INT64_MAX) lam = INT64_MAX;
  return (int64_t)lam;
}

bool lazy_block_ok(uint64_t p, int u, int v, int64_t L) {
  // A block starts from a value in [-p, 2p - 1] and adds L non-negative
  // terms, each at most w: every partial sum stays in [-p, 2^t] if
  // L w + 2p - 1 <= 2^t.
  u128 w = word_product_bound(p, u, v);
  return (u128)L * w + 2 * (u128)p - 1 <= (u128)kTwoT;
}

namespace {

// Relative cost per real k-term of one 16x16 output tile, in SIMD cycles,
// measured shape of the gfx950 pipes: an FP64 16x16x4 MFMA issues every 64
// cycles and FP64 VALU instructions (4 cycles each) do not overlap with it.
// An in-loop reduction of a 16x16 tile is 4 values per lane: 3 VALU ops
// each when correction-free, about 11 with Alg. 1's two corrections.
double block_cost(int S, int64_t L, bool lazy) {
  const double mfma = 64.0 * (S / 4);
  const double red = lazy ? 4 * 3 * 4.0 : 4 * 11 * 4.0;
  return (mfma + red) / (double)L;
}

struct KBlock {
  int64_t L;
  int S;
  bool lazy;
  bool extended;
  double cost;
  bool biased;  // the in-loop reduction is the biased one (range [-2^t, -2^t + 4p))
};

// Correction-free reduction for a block of L terms within the paper's
// bound: the plain form when a block started in [-p, 2p) stays within 2^t,
// else the biased form when a block started in [-2^t, -2^t + 4p) stays
// within [-2^t, 2^t].  The block length is the paper's either way; only the
// range the accumulator restarts from differs.  Returns false (full Alg. 1
// in the loop) when neither holds or strict reductions are asked for.
bool correction_free(uint64_t p, int u, int v, int64_t L, bool strict, bool* biased) {
  *biased = false;
  if (strict) return false;
  if (lazy_block_ok(p, u, v, L)) return true;
  if (extended_block_ok(p, u, v, L)) {
    *biased = true;
    return true;
  }
  return false;
}

// Best (L, S) for one word pair.  Paper mode: L <= the paper's lambda, a
// correction-free reduction where correction_free allows one.  With extended
// allowed, blocks under the extended bound compete too (biased reduction);
// near p = 2^(t-1) that bound is the smaller one and the paper mode wins.
// Centered words: L <= centered_lambda, always the one-step reduction.
KBlock choose_kblock(uint64_t p, int u, int v, int64_t k, bool strict, bool allow_extended,
                     bool centered = false) {
  KBlock best{0, 0, false, false, 1e300, false};
  const int64_t lam_paper = centered ? centered_lambda(p, u, v) : paper_lambda(p, u, v);
  const int64_t lam_ext = allow_extended ? extended_lambda(p, u, v) : 0;
  auto consider = [&](int S, int64_t L, bool ext) {
    if (L < 1 || L > (ext ? lam_ext : lam_paper)) return;
    bool biased = ext;
    const bool lazy = centered || ext || correction_free(p, u, v, L, strict, &biased);
    double c = block_cost(S, L, lazy);
    // a block longer than k never reduces in the loop: cost of the MFMAs only
    if (L >= k && k > 0) c = 64.0 * (S / 4) / (double)L;
    if (c < best.cost - 1e-12) best = {L, S, lazy, ext, c, biased};
  };
  for (int e = 0; e < (allow_extended ? 2 : 1); e++) {
    const bool ext = e == 1;
    const int64_t lambda = ext ? lam_ext : lam_paper;
    for (int S : {4, 8, 16}) consider(S, lambda < S ? lambda : S, ext);
    // longer blocks of whole k-steps, no zero slots: L = S = 4 j >= 12
    // (the kernel counts k-steps, so a block may end inside a stage)
    const int64_t cap = (int64_t)1 << 26;  // beyond this the in-loop cost is nil
    const int64_t L4 = std::min<int64_t>(lambda, cap) / 4 * 4;
    if (L4 >= 12 && L4 != kBK) consider((int)L4, L4, ext);
  }
  return best;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Seconds for the FP64-word kernel: cycles per 16x16 output tile per k-term
// (block_cost) over 1024 SIMDs at 2.4 GHz.
double fp64_seconds(int64_t m, int64_t n, int64_t k, int uv, double cost) {
  const double tiles = (double)cdiv(m, 16) * (double)cdiv(n, 16);
  return tiles * (double)k * cost * uv / (1024.0 * 2.4e9);
}

// Seconds for the INT8-digit form: D^2 digit GEMMs at an assumed 60% of the
// 5 POP/s INT8 peak, two digitizing passes over A and B (8 bytes read, D
// written per entry, 70% of 8 TB/s), the binary64 folds (about 25 VALU
// operations per digit weight per output and fold) and three launches.
double int8_seconds(int64_t m, int64_t n, int64_t k, int d) {
  const double kp = (double)cdiv(k, 64) * 64.0;
  const double gemm = (double)d * d * 2.0 * m * n * kp / (0.6 * 5.0e15);
  const double digitize = (8.0 + d) * ((double)m * k + (double)k * n) / (0.7 * 8.0e12);
  const double folds = (double)cdiv(k, int8_kblock(d));
  const double fold = (2.0 * d - 1) * 25.0 * (double)m * n * folds / (64.0 * 1024.0 * 2.4e9 / 4.0);
  return gemm + digitize + fold + 3 * 4e-6;
}

// Among the tiles that fill the chip (two workgroups per CU, counting the
// k-ranges split-K adds for long k), the one with the least padded output
// area, the larger on a tie (a 128-wide tile on n = 32 would compute 75%
// padding); if none fills the chip, the smallest.
int pick_tile(int u, int v, int64_t m, int64_t n, int64_t stages, int slots, int64_t kblock) {
  int best = 0;
  int64_t best_area = 0;
  for (int id = 1; id <= 3; id++) {
    Fp64Tile t = fp64_tile(id, u, v, slots, kblock);
    const int64_t bm = fp64_bm(t), bn = fp64_bn(t);
    const int64_t nb = cdiv(m, bm) * cdiv(n, bn);
    if (nb * choose_splits(nb, stages, 64) < 512) continue;
    const int64_t area = cdiv(m, bm) * bm * cdiv(n, bn) * bn;
    if (best == 0 || area < best_area) {
      best = id;
      best_area = area;
    }
  }
  return best ? best : 3;
}

// ---------------------------------------------------------------- tuning cache
// Fastest measured plan per (bitsize of p, ceil(log2) of m, n, k, bound mode:
// 0 paper, 1 extended allowed, 2 centered words); filled by mmp_autotune,
// read by AUTO plans.  The file field "ext" holds the mode.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, TunedChoice> g_tune;

int log2_ceil(int64_t x) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) b++;
  return b;
}

}  // namespace

std::tuple<int, int, int, int, int> tune_key(uint64_t p, int64_t m, int64_t n, int64_t k, int mode) {
  int bits = 0;
  while (bits < 64 && (p >> bits) != 0) bits++;
  return std::make_tuple(bits, log2_ceil(m), log2_ceil(n), log2_ceil(k), mode);
}

void tune_store(uint64_t p, int64_t m, int64_t n, int64_t k, int mode, const TunedChoice& c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[tune_key(p, m, n, k, mode)] = c;
}

bool tune_lookup(uint64_t p, int64_t m, int64_t n, int64_t k, int mode, TunedChoice* c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(p, m, n, k, mode));
  if (it == g_tune.end()) return false;
  *c = it->second;
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

int tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return MMP_EINVAL;
  std::fprintf(f, "{\"entries\": [\n");
  size_t i = 0;
  for (auto& kv : g_tune) {
    const auto& k = kv.first;
    const TunedChoice& c = kv.second;
    std::fprintf(f,
                 "  {\"bits\": %d, \"lm\": %d, \"ln\": %d, \"lk\": %d, \"ext\": %d, \"form\": %d, \"u\": %d, "
                 "\"v\": %d, \"tile\": %d, \"kblock\": %lld, \"ms\": %.6f}%s\n",
                 std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), c.form, c.u, c.v,
                 c.tile, (long long)c.kblock, c.ms, ++i < g_tune.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return MMP_OK;
}

int tune_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return MMP_ENOTFOUND;
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof line, f)) {
    int bits, lm, ln, lk, ext, form, u, v, tile;
    long long kb;
    double ms;
    if (std::sscanf(line,
                    " {\"bits\": %d, \"lm\": %d, \"ln\": %d, \"lk\": %d, \"ext\": %d, \"form\": %d, \"u\": %d, "
                    "\"v\": %d, \"tile\": %d, \"kblock\": %lld, \"ms\": %lf",
                    &bits, &lm, &ln, &lk, &ext, &form, &u, &v, &tile, &kb, &ms) == 11) {
      std::lock_guard<std::mutex> lk2(g_tune_mu);
      g_tune[std::make_tuple(bits, lm, ln, lk, ext)] = TunedChoice{form, u, v, tile, (int64_t)kb, ms};
      n++;
    }
  }
  std::fclose(f);
  return n;
}

int digits_for(uint64_t p) {
  int bits = 0;
  while (bits < 64 && (p >> bits) != 0) bits++;
  return (bits + 7) / 8;
}

int default_splits(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k) {
  if (pl.form == MMP_FORM_INT8_WORDS) return choose_splits_fill(cdiv(m, 64) * cdiv(n, 64), cdiv(k, 64), 32);
  // real k-terms per 16-slot stage: fewer only when blocks leave zero slots
  const int64_t KR = (pl.slots <= kBK && pl.kblock < pl.slots) ? (kBK / pl.slots) * pl.kblock : kBK;
  return choose_splits(cdiv(m, pl.bm) * cdiv(n, pl.bn), cdiv(k, KR), 64);
}

int64_t int8_kblock(int digits) {
  // K D 2^14 <= 2^31 - 1 keeps every int32 accumulator exact for any
  // entries (|d_i d_j| <= 2^14); int8_bound_* give the longer block that the
  // entries' actual digit range allows
  const int64_t K = ((int64_t)1 << 31) - 1;
  const int64_t per = (int64_t)digits << 14;
  return (K / per) / 64 * 64;
}

// ---- exact int32 block of the digit GEMM ------------------------------------
// The digit GEMM sees every entry as an integer x' in an interval [lo, hi] of
// [-128 R, 127 R], R = (256^D - 1) / 255, written with D signed digits in
// [-128, 127] (the low byte read as int8, then the exact carry).  Because
// the digit set is 256 consecutive integers and 255 R < 256^D, values are
// ordered like their digit vectors read from the top digit down, so the
// digit vectors of [lo, hi] form a union of at most 2D + 1 boxes (a common
// top prefix, one digit in a sub-range, the digits below it free).  One
// k-term adds sum_{i+j=s} a_i b_j to the accumulator of weight s; within a
// pair of boxes every a_i meets exactly one b_j, so the extremes over the
// pair are sums of the extremes of single products over the digits' ranges,
// which sit at range ends.  A block of K k-terms is then exact when
// K tmax <= 2^31 - 1 and K (-tmin) <= 2^31.
namespace {

struct DigitBox {
  int lo[8], hi[8];
};

void signed_digits(__int128 v, int D, int (&d)[8]) {
  for (int i = 0; i < D; i++) {
    const int di = (int)(int8_t)(uint8_t)(v & 0xff);
    d[i] = di;
    v = (v - di) >> 8;
  }
}

int digit_boxes(int D, int64_t lo, int64_t hi, DigitBox* out) {
  int L[8], H[8];
  signed_digits(lo, D, L);
  signed_digits(hi, D, H);
  int t = D - 1;
  while (t >= 0 && L[t] == H[t]) t--;
  int nb = 0;
  auto fixed = [&](const int* P, int above, DigitBox& b) {  // digits >= above follow P
    for (int i = above; i < D; i++) b.lo[i] = b.hi[i] = P[i];
    for (int i = 0; i < above; i++) {
      b.lo[i] = -128;
      b.hi[i] = 127;
    }
  };
  if (t < 0) {  // lo == hi
    fixed(L, 0, out[nb++]);
    return nb;
  }
  if (L[t] + 1 <= H[t] - 1) {  // digit t strictly between the ends
    DigitBox& b = out[nb++];
    fixed(L, t, b);
    b.lo[t] = L[t] + 1;
    b.hi[t] = H[t] - 1;
  }
  // digit t = L[t]: the lower digits at or above lo's, by the first one that
  // exceeds lo's; then lo itself
  for (int j = t - 1; j >= 0; j--) {
    if (L[j] == 127) continue;
    DigitBox& b = out[nb++];
    fixed(L, j, b);
    b.lo[j] = L[j] + 1;
    b.hi[j] = 127;
  }
  fixed(L, 0, out[nb++]);
  // digit t = H[t]: the lower digits at or below hi's; then hi itself
  for (int j = t - 1; j >= 0; j--) {
    if (H[j] == -128) continue;
    DigitBox& b = out[nb++];
    fixed(H, j, b);
    b.lo[j] = -128;
    b.hi[j] = H[j] - 1;
  }
  fixed(H, 0, out[nb++]);
  return nb;
}

__int128 digits_value(const int (&d)[8], int D) {
  __int128 v = 0;
  for (int i = D - 1; i >= 0; i--) v = v * 256 + d[i];
  return v;
}

}  // namespace

int64_t radix_top(int D) {  // 127 R: the largest value D signed digits hold
  int64_t top = 0;
  for (int i = 0; i < D; i++) top = top * 256 + 127;
  return top;
}

Int8Bound int8_bound_interval(int D, int64_t lo, int64_t hi) {
  Int8Bound r;
  std::memset(&r, 0, sizeof(r));
  r.digits = D;
  r.lo = lo;
  r.hi = hi;
  DigitBox boxes[17];
  const int nb = digit_boxes(D, lo, hi, boxes);
  bool first = true;
  for (int s = 0; s <= 2 * D - 2; s++) {
    for (int ba = 0; ba < nb; ba++) {
      for (int bb = 0; bb < nb; bb++) {
        const DigitBox& A = boxes[ba];
        const DigitBox& B = boxes[bb];
        int64_t smax = 0, smin = 0;
        int amax[8], bmax[8], amin[8], bmin[8];
        for (int i = 0; i < D; i++) {
          amax[i] = amin[i] = A.lo[i];
          bmax[i] = bmin[i] = B.lo[i];
        }
        for (int i = std::max(0, s - D + 1); i <= std::min(s, D - 1); i++) {
          const int j = s - i;
          const int ea[2] = {A.lo[i], A.hi[i]}, eb[2] = {B.lo[j], B.hi[j]};
          int64_t hi_ = INT64_MIN, lo_ = INT64_MAX;
          for (int x = 0; x < 2; x++)
            for (int y = 0; y < 2; y++) {
              const int64_t pr = (int64_t)ea[x] * eb[y];
              if (pr > hi_) {
                hi_ = pr;
                amax[i] = ea[x];
                bmax[j] = eb[y];
              }
              if (pr < lo_) {
                lo_ = pr;
                amin[i] = ea[x];
                bmin[j] = eb[y];
              }
            }
          smax += hi_;
          smin += lo_;
        }
        if (first || smax > r.term_max) {
          r.term_max = smax;
          r.weight_max = s;
          r.witness_max[0] = (int64_t)digits_value(amax, D);
          r.witness_max[1] = (int64_t)digits_value(bmax, D);
        }
        if (first || smin < r.term_min) {
          r.term_min = smin;
          r.weight_min = s;
          r.witness_min[0] = (int64_t)digits_value(amin, D);
          r.witness_min[1] = (int64_t)digits_value(bmin, D);
        }
        first = false;
      }
    }
  }
  // the longest block of whole 64-term stages within int32 at both ends
  int64_t K = INT64_MAX;
  if (r.term_max > 0) K = std::min<int64_t>(K, (((int64_t)1 << 31) - 1) / r.term_max);
  if (r.term_min < 0) K = std::min<int64_t>(K, ((int64_t)1 << 31) / -r.term_min);
  if (K == INT64_MAX) K = (int64_t)1 << 40;  // all-zero entries: any block is exact
  r.kblock = K / 64 * 64;
  return r;
}

// Residues mod p as the digitizer maps them: x' = x, or x - p when x exceeds
// 127 R, with D = ceil(bitsize(p) / 8), so x' lies in [127 R + 1 - p, 127 R]
// (or [0, p - 1] when p - 1 <= 127 R).
Int8Bound int8_bound_residues(uint64_t p) {
  const int D = digits_for(p);
  const int64_t top = radix_top(D);
  const int64_t pm1 = (int64_t)p - 1;
  return int8_bound_interval(D, pm1 > top ? top + 1 - (int64_t)p : 0, std::min(pm1, top));
}

// Integers of the multi-modular product: [0, 2^entry_bits - 1] as they are
// (computed once per width).
Int8Bound int8_bound_integers(int entry_bits) {
  static std::mutex mu;
  static Int8Bound cache[64];
  static bool have[64] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!have[entry_bits]) {
    const int D = crt_digits(entry_bits);
    cache[entry_bits] = int8_bound_interval(D, 0, (int64_t)((((uint64_t)1) << entry_bits) - 1));
    have[entry_bits] = true;
  }
  return cache[entry_bits];
}

// The fewest signed base-256 digits that hold every value below 2^entry_bits:
// 2^entry_bits - 1 <= 127 R (at most 8 for entry_bits <= 62).
int crt_digits(int entry_bits) {
  const uint64_t vmax = (((uint64_t)1) << entry_bits) - 1;
  int D = 1;
  while (D < 8 && (uint64_t)radix_top(D) < vmax) D++;
  return D;
}

size_t int8_workspace_bytes(int digits, int64_t m, int64_t n, int64_t k) {
  const int64_t kp = cdiv(k, 64) * 64;
  return digit_planes_bytes(digits, m, kp) + digit_planes_bytes(digits, n, kp);
}

size_t int8_planes_bytes(int digits, int64_t m, int64_t n, int64_t k, bool res_a, bool res_b) {
  const int64_t kp = cdiv(k, 64) * 64;
  const size_t bytes = (res_a ? 0 : digit_planes_bytes(digits, m, kp)) + (res_b ? 0 : digit_planes_bytes(digits, n, kp));
  return (bytes + 255) / 256 * 256;
}

static int plan_impl(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const mmp_opts* opts,
                     mmp_plan_t* out, bool use_tuned) {
  if (!out) return MMP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  mmp_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (opts) {
    if (opts->batch_launch < 0 || opts->batch_launch > 2) return MMP_EINVAL;
    // prepared operands are taken by mm_modp_async alone, which plans without them
    if (opts->prepared_a || opts->prepared_b) return MMP_EINVAL;
  }
  if (p < 5 || p >= kPMax) return MMP_EINVAL;
  if (m < 0 || n < 0 || k < 0) return MMP_EINVAL;
  if ((u == 0) != (v == 0)) return MMP_EINVAL;
  if (u != 0 && !supported_words(u, v)) return MMP_EINVAL;
  if (o.form != MMP_FORM_AUTO && o.form != MMP_FORM_FP64_WORDS && o.form != MMP_FORM_INT8_WORDS)
    return MMP_EINVAL;
  if (o.force_kblock < 0 || o.tile < 0 || o.tile > 3 || o.splits < 0 || o.splits > 64) return MMP_EINVAL;

  const bool strict = o.strict_fmod != 0;
  const bool extended = o.extended_block != 0;
  const bool centered = o.centered_words != 0;
  if (extended && strict) return MMP_EINVAL;  // the extended range needs the biased reduction
  if (extended && o.form == MMP_FORM_INT8_WORDS) return MMP_EINVAL;
  if (centered && (extended || strict || o.form == MMP_FORM_INT8_WORDS)) return MMP_EINVAL;

  // INT8-digit form: asked for, or chosen by cost when neither the words
  // nor the block are forced.
  const int d8 = digits_for(p);
  auto plan_int8 = [&]() {
    out->p = p;
    out->u = 0;
    out->v = 0;
    out->form = MMP_FORM_INT8_WORDS;
    out->digits_a = d8;
    out->digits_b = d8;
    // the exact block of these entries (int8_bound_residues) matters only
    // when k exceeds the block any entries allow; shorter products run whole
    // k as one block either way, and skip the bound's cost (about 0.1 ms)
    out->kblock_int8 = int8_kblock(d8);
    if (k > out->kblock_int8) out->kblock_int8 = int8_bound_residues(p).kblock;
    out->q = 1.0 / (double)p;
    out->bk = 64;
    out->est_seconds = int8_seconds(m, n, k, d8);
    out->splits = o.splits ? o.splits : default_splits(*out, m, n, k);
    out->workspace_bytes = (int8_workspace_bytes(d8, m, n, k) + 255) / 256 * 256;
    if (out->splits > 1) out->workspace_bytes += 8 * (size_t)out->splits * (size_t)m * (size_t)n;
    return MMP_OK;
  };
  if (o.form == MMP_FORM_INT8_WORDS) {
    if (u != 0 || o.tile != 0) return MMP_EINVAL;
    int st = plan_int8();
    if (o.force_kblock != 0) {  // a shorter int32 block, whole 64-term stages
      if (o.force_kblock % 64 != 0) return MMP_EINVAL;
      if (o.force_kblock > out->kblock_int8) return MMP_EBOUND;
      out->kblock_int8 = o.force_kblock;
    }
    return st;
  }

  // Candidate word pairs.  With u = v = 0 the planner takes the cheapest by
  // the cost model (uv word products, each at its own block cost), which
  // reproduces the bitsize ranges after Table tab.summary; ties go to the
  // orientation that puts extra words on the operand with the smaller outer
  // dimension (the concatenation rule of Section 3.2).
  // A tuned choice for this class of products, if mmp_autotune measured one.
  if (use_tuned && o.form == MMP_FORM_AUTO && u == 0 && o.force_kblock == 0 && o.tile == 0) {
    TunedChoice c;
    if (tune_lookup(p, m, n, k, centered ? 2 : extended ? 1 : 0, &c)) {
      mmp_opts o2 = o;
      o2.form = c.form;
      o2.tile = c.form == MMP_FORM_FP64_WORDS ? c.tile : 0;
      o2.force_kblock = c.form == MMP_FORM_FP64_WORDS ? c.kblock : 0;
      const int st = plan_impl(p, c.form == MMP_FORM_FP64_WORDS ? c.u : 0, c.form == MMP_FORM_FP64_WORDS ? c.v : 0,
                               m, n, k, &o2, out, false);
      if (st == MMP_OK) return MMP_OK;  // else the tuned block does not fit this p: plan afresh
    }
  }
  static const int cand[][2] = {{1, 1}, {1, 2}, {2, 1}, {1, 3}, {3, 1}, {2, 2},
                                {1, 4}, {4, 1}, {2, 3}, {3, 2}, {2, 4}, {4, 2}};
  int bu = u, bv = v;
  KBlock bk{};
  if (u == 0) {
    double best = 1e300;
    for (auto& c : cand) {
      int cu = c[0], cv = c[1];
      if (n < m && cu > cv) continue;  // words on B when B is the narrower side
      if (n > m && cv > cu) continue;
      if ((centered ? centered_lambda(p, cu, cv) : paper_lambda(p, cu, cv)) < 1) continue;
      KBlock kb = choose_kblock(p, cu, cv, k, strict, extended, centered);
      double cost = kb.cost * cu * cv;
      if (cost < best * (1 - 1e-9)) {
        best = cost;
        bu = cu;
        bv = cv;
        bk = kb;
      }
    }
    if (best >= 1e299) return MMP_EBOUND;
  }
  const int64_t lambda = paper_lambda(p, bu, bv);
  const int64_t lam_c = centered ? centered_lambda(p, bu, bv) : 0;
  if (centered ? lam_c < 1 : lambda < 1) return MMP_EBOUND;
  if (o.force_kblock > 0) {
    int64_t L = o.force_kblock;
    // a forced block takes the paper's bound when it fits, else the extended
    // one; with centered words, the centered bound
    const bool ext = !centered && L > lambda;
    if (centered && L > lam_c) return MMP_EBOUND;
    if (ext && (!extended || L > extended_lambda(p, bu, bv))) return MMP_EBOUND;
    int S;
    if (L <= 4) S = 4;
    else if (L <= 8) S = 8;
    else if (L <= kBK) S = kBK;
    else if (L % 4 == 0) S = (int)L;
    else return MMP_EINVAL;  // longer blocks must be whole MFMA k-steps
    if (L > ((int64_t)1 << 26)) return MMP_EINVAL;
    bool biased = ext;
    const bool lazy = centered || ext || correction_free(p, bu, bv, L, strict, &biased);
    bk = {L, S, lazy, ext, block_cost(S, L, lazy), biased && !centered};
  } else if (u != 0) {
    bk = choose_kblock(p, bu, bv, k, strict, extended, centered);
  }

  out->p = p;
  out->u = bu;
  out->v = bv;
  out->form = MMP_FORM_FP64_WORDS;
  out->alpha = iroot_ceil(p, bu);
  out->beta = iroot_ceil(p, bv);
  out->lambda = lambda;
  out->kblock = bk.L;
  out->slots = bk.S;
  out->lazy = bk.lazy ? 1 : 0;
  out->extended = bk.extended ? 1 : 0;
  out->biased = bk.biased && !centered ? 1 : 0;
  out->centered = centered ? 1 : 0;
  const int64_t KR = (bk.S <= kBK && bk.L < bk.S) ? (kBK / bk.S) * bk.L : kBK;  // real k-terms per stage
  out->tile = o.tile ? o.tile : pick_tile(bu, bv, m, n, cdiv(k, KR), bk.S, bk.L);
  Fp64Tile t = fp64_tile(out->tile, bu, bv, bk.S, bk.L);
  out->bm = fp64_bm(t);
  out->bn = fp64_bn(t);
  out->bk = kBK;
  out->q = 1.0 / (double)p;
  out->est_seconds = fp64_seconds(m, n, k, bu * bv, bk.cost);
  out->splits = o.splits ? o.splits : default_splits(*out, m, n, k);
  out->workspace_bytes = out->splits > 1 ? 8 * (size_t)out->splits * (size_t)m * (size_t)n : 0;
  if (o.form == MMP_FORM_AUTO && u == 0 && o.force_kblock == 0 && o.tile == 0 && !extended && !centered &&
      int8_seconds(m, n, k, d8) < out->est_seconds) {
    std::memset(out, 0, sizeof(*out));
    return plan_int8();
  }
  return MMP_OK;
}

int plan(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const mmp_opts* opts, mmp_plan_t* out) {
  return plan_impl(p, u, v, m, n, k, opts, out, true);
}

}  // namespace mmp
