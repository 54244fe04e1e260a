// Internal declarations shared by the planner, the C-ABI layer and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include "mmp.h"

namespace mmp {

constexpr int kT = 53;                              // binary64 significand bits
constexpr uint64_t kTwoT = 1ull << kT;              // 2^t
constexpr uint64_t kPMax = 1ull << (kT - 1);        // p < 2^(t-1)  (Alg. 1)
constexpr int kMaxWords = 4;                        // u, v <= 4
constexpr int kMaxWordProducts = 8;                 // u v <= 8
constexpr int kBK = 16;                             // k-slots per LDS stage (FP64 form)

// FP64-form tile shapes.  A workgroup is 4 waves in a 2 x 2 grid; each wave
// owns TM x TN MFMA tiles of 16 x 16 outputs for every word pair.
struct Fp64Tile {
  int tm, tn;
};

// tile id 1 (large), 2 (medium), 3 (small) for a given number of word products.
// Accumulator VGPRs per lane = uv * tm * tn * 8 (a 16x16 FP64 tile is 4
// values of 2 VGPRs per lane); the shapes keep that at 96..128.
constexpr Fp64Tile fp64_tile_c(int tile_id, int uv) {
  return tile_id == 3   ? Fp64Tile{1, 1}
         : tile_id == 2 ? (uv <= 2 ? Fp64Tile{2, 2} : uv <= 4 ? Fp64Tile{1, 2} : Fp64Tile{1, 1})
                        : (uv == 1   ? Fp64Tile{4, 4}
                           : uv == 2 ? Fp64Tile{2, 4}
                           : uv <= 4 ? Fp64Tile{2, 2}
                                     : Fp64Tile{1, 2});
}
inline Fp64Tile fp64_tile(int tile_id, int uv) { return fp64_tile_c(tile_id, uv); }
inline int fp64_bm(const Fp64Tile& t) { return 2 * 16 * t.tm; }
inline int fp64_bn(const Fp64Tile& t) { return 2 * 16 * t.tn; }

// Exact integer helpers (host).
uint64_t iroot_ceil(uint64_t p, int u);        // smallest a with a^u >= p
int64_t paper_lambda(uint64_t p, int u, int v);  // eq. lambda-sw / eq. cAcB, 0 if none
// True when a k-block of L terms may start anywhere in [-p, 2p) (the range a
// correction-free reduction leaves) and stay within 2^t.
bool lazy_block_ok(uint64_t p, int u, int v, int64_t L);
bool supported_words(int u, int v);

int plan(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const mmp_opts* opts,
         mmp_plan_t* out);

// Kernel arguments for the FP64-word form.
struct Fp64Args {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k, lda, ldb, ldc;
  double p, q, alpha, beta, ainv, binv;  // ainv/binv: exact 1/alpha, 1/beta when powers of two, else 0
  int L;           // real k-terms per block
  int S;           // k-slots per block (S >= L; zeros fill the rest)
  int KR;          // real k-terms per LDS stage
  int stages_per_block;  // S >= 16: LDS stages per block (S / 16)
  int lazy;              // in-loop reductions without corrections
};

// INT8-digit form: digit planes in a device workspace, then the digit GEMM.
constexpr int kMaxDigits = 7;  // signed base-256 digits cover p < 2^56
struct Int8Args {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k, lda, ldb, ldc;
  int64_t kp;        // k rounded up to a multiple of 64 (zero digits beyond k)
  uint64_t p;
  double q;
  int64_t kblock;    // k-terms per int32 accumulation block (multiple of 64)
  int8_t* work;      // D (m + n) kp bytes
};
int digits_for(uint64_t p);                       // ceil(bitsize(p) / 8)
int64_t int8_kblock(int digits);                  // exact-int32 block length
size_t int8_workspace_bytes(int digits, int64_t m, int64_t n, int64_t k);
int launch_int8_digits(int digits, const Int8Args& a, void* stream);

// Launch the fused FP64-word kernel; returns a hipError_t value (0 = success).
int launch_fp64_words(int u, int v, int tile_id, const Fp64Args& a, void* stream);
// Fill a row-major m x n matrix (leading dimension ld) with +0.0.
int launch_zero_fill(double* C, int64_t m, int64_t n, int64_t ld, void* stream);
// Scan for entries outside [0, p) or non-integral; sets *flag (device int) nonzero.
int launch_validate(const double* X, int64_t rows, int64_t cols, int64_t ld, double p, int* flag,
                    void* stream);

}  // namespace mmp
