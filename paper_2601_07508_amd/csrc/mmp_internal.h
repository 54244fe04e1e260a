// Internal declarations shared by the planner, the C-ABI layer and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "mmp.h"

namespace mmp {

constexpr int kT = 53;                              // binary64 significand bits
constexpr uint64_t kTwoT = 1ull << kT;              // 2^t
constexpr uint64_t kPMax = 1ull << (kT - 1);        // p < 2^(t-1)  (Alg. 1)
constexpr int kMaxWords = 4;                        // u, v <= 4
constexpr int kMaxWordProducts = 8;                 // u v <= 8
constexpr int kBK = 16;                             // k-slots per LDS stage (FP64 form)
constexpr int kMaxBatch = 16;                       // products per batched launch

// FP64-form tile shapes.  A workgroup is 4 waves in a 2 x 2 grid; each wave
// owns TM x TN MFMA tiles of 16 x 16 outputs for every word pair.
struct Fp64Tile {
  int tm, tn;
};

// tile id 1 (large), 2 (medium), 3 (small) for a given number of word products.
// Accumulator VGPRs per lane = uv * tm * tn * 8 (a 16x16 FP64 tile is 4
// values of 2 VGPRs per lane); the shapes keep that at 96..128.
// Tile 1, the large shape, keeps each word pair within 256 VGPRs and two
// workgroups per CU (LDS): the longer side goes to the operand with fewer
// words, whose fragments are the cheaper ones to hold.
// wide: the kernel class reduces only every whole number of k-steps >= 3
// and has no padded stages (fewer live registers), which lets (1,1) take
// 4 x 4 tiles.
constexpr Fp64Tile fp64_tile_c(int tile_id, int u, int v, bool wide) {
  if (tile_id == 3) return Fp64Tile{1, 1};
  if (tile_id == 2) return Fp64Tile{2, 1};  // 64 x 32: narrow outputs (n <= 32) and mid-size products
  if (u == 1 && v == 1) return wide ? Fp64Tile{4, 4} : Fp64Tile{4, 2};
  if (u * v == 2) return u < v ? Fp64Tile{4, 2} : Fp64Tile{2, 4};
  if (u == 1 && v == 4) return Fp64Tile{4, 1};
  if (u == 4 && v == 1) return Fp64Tile{1, 4};
  if (u * v <= 4) return Fp64Tile{2, 2};  // (1,3), (3,1), (2,2)
  return u >= v ? Fp64Tile{1, 2} : Fp64Tile{2, 1};
}
inline bool fp64_wide(int slots, int64_t kblock) { return slots > 8 && !(slots <= 16 && kblock < slots); }
inline Fp64Tile fp64_tile(int tile_id, int u, int v, int slots, int64_t kblock) {
  return fp64_tile_c(tile_id, u, v, fp64_wide(slots, kblock));
}
inline int fp64_bm(const Fp64Tile& t) { return 2 * 16 * t.tm; }
inline int fp64_bn(const Fp64Tile& t) { return 2 * 16 * t.tn; }

// Exact integer helpers (host).
uint64_t iroot_ceil(uint64_t p, int u);        // smallest a with a^u >= p
int64_t paper_lambda(uint64_t p, int u, int v);  // eq. lambda-sw / eq. cAcB, 0 if none
// True when a k-block of L terms may start anywhere in [-p, 2p) (the range a
// correction-free reduction leaves) and stay within 2^t.
bool lazy_block_ok(uint64_t p, int u, int v, int64_t L);
bool supported_words(int u, int v);
// The extended bound: a block started in [-2^t, -2^t + 4p) (the biased
// reduction's range) stays within [-2^t, 2^t].
bool extended_block_ok(uint64_t p, int u, int v, int64_t L);
int64_t extended_lambda(uint64_t p, int u, int v);
// Centered words: largest |word| of an entry split into u words, and the
// longest block whose partial sums stay within 2^t from the centered
// reduction's range.
uint64_t centered_word_bound(uint64_t p, int u);
bool centered_block_ok(uint64_t p, int u, int v, int64_t L);
int64_t centered_lambda(uint64_t p, int u, int v);

int plan(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const mmp_opts* opts,
         mmp_plan_t* out);

// Tuning cache (mmp_autotune fills it; AUTO plans read it).
struct TunedChoice {
  int form, u, v, tile;
  int64_t kblock;
  double ms;
};
void tune_store(uint64_t p, int64_t m, int64_t n, int64_t k, int mode, const TunedChoice& c);
bool tune_lookup(uint64_t p, int64_t m, int64_t n, int64_t k, int mode, TunedChoice* c);
void tune_clear();
int tune_save(const char* path);
int tune_load(const char* path);
// Fill X (count binary64 values) with a hash of the index mod p (scratch inputs).
int launch_fill_mod(double* X, int64_t count, uint64_t p, uint64_t seed, void* stream);

// Kernel arguments for the FP64-word form.
struct Fp64Args {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k, lda, ldb, ldc;
  double p, q, alpha, beta, ainv, binv;  // ainv, binv: fl(1/alpha), fl(1/beta)
  int afix, bfix;        // 1: the base is not a power of two, so a split quotient needs its correction step
  int L;           // real k-terms per block
  int S;           // k-slots per block (S >= L; zeros fill the rest)
  int KR;          // real k-terms per LDS stage
  int ksteps_per_block;  // S / 4: MFMA k-steps per block (S >= 12 or a padded 16-slot stage)
  int lazy;              // in-loop reductions without corrections
  double bias;           // K in the in-loop reduction c = floor(x q + K) (0, or floor(2^t / p) - 1)
  double acc_init;       // accumulator start value: -K p (congruent to 0)
  int splits;            // split-K: k-ranges of this product (1: none)
  double* partial;       // splits > 1: residues per k-range, [splits][m][n]
  int centered;          // centered words: x - p when 2x > p, round-to-nearest splits
};

// INT8-digit form: digit planes in a device workspace, then the digit GEMM.
constexpr int kMaxDigits = 7;  // signed base-256 digits cover p < 2^56
// A digit plane of `rows` rows by kp k-bytes (kp a multiple of 64) is stored
// in blocks of 16 rows by 64 k-bytes, 1 KB each, row-major inside a block:
// byte (r, c) sits at (r / 16) 16 kp + (c / 64) 1024 + (r % 16) 64 + c % 64.
// One block is what the digit GEMM copies into LDS in one instruction, and a
// 16-row group's successive k-stages are contiguous.  A plane takes
// plane_rows(rows) kp bytes; rows past `rows` in the last block are never
// written or read.
inline int64_t plane_rows(int64_t rows) { return (rows + 15) / 16 * 16; }
inline size_t digit_planes_bytes(int digits, int64_t rows, int64_t kp) {
  return (size_t)digits * (size_t)plane_rows(rows) * (size_t)kp;
}
struct Int8Args {
  const double* A;
  const double* B;
  double* C;
  int64_t m, n, k, lda, ldb, ldc;
  int64_t kp;        // k rounded up to a multiple of 64 (zero digits beyond k)
  uint64_t p;
  double q;
  int64_t kblock;    // k-terms per int32 accumulation block (multiple of 64)
  int8_t* work;      // planes of A (digit_planes_bytes(D, m, kp)), then of B^T
  const int8_t* resident_a;  // optional ready planes of A (then A is not digitised)
  const int8_t* resident_b;  // optional ready planes of B^T
  // work holds the planes made per call: A's (absent when resident), then B's
  int splits;                // split-K: k-ranges (1: none)
  double* partial;           // splits > 1: residues per k-range, [splits][m][n]
};
// C = sum over the splits of partial[s] mod p (each partial in [0, p)).
int launch_splitk_reduce(const double* partial, int splits, int64_t m, int64_t n, double p, double* C, int64_t ldc,
                         void* stream);
// Split count for a product of `tiles` output tiles and `stages` k-stages.
int choose_splits(int64_t tiles, int64_t stages, int64_t min_stages_per_split);
int choose_splits_fill(int64_t tiles, int64_t stages, int64_t min_stages_per_split);  // INT8 digit GEMM
// the planner's split-K for a plan (its form, tile and block) and shape
int default_splits(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k);
// Digit planes of one operand side into out (side 0: A's rows, D planes of
// rows x kp; side 1: B's columns, D planes of cols x kp; blocked as above).
int launch_int8_digitize_side(int digits, int side, const double* X, int64_t rows, int64_t cols, int64_t ld,
                              int64_t kp, uint64_t p, int8_t* out, void* stream);
int digits_for(uint64_t p);                       // ceil(bitsize(p) / 8)
int64_t int8_kblock(int digits);                  // exact-int32 block length for any entries
// The exact int32 block for the entries' actual digit range: the extremes of
// one k-term's digit-weight sum, entries reaching them, and the longest block
// of whole 64-term stages that keeps every accumulator in int32.
struct Int8Bound {
  int digits, weight_max, weight_min;
  int64_t lo, hi;                  // digit values x' of the entries lie in [lo, hi]
  int64_t term_max, term_min;      // extremes of sum_{i+j=s} a_i b_j for one k-term
  int64_t witness_max[2], witness_min[2];  // values (a, b) in [lo, hi] reaching them
  int64_t kblock;
};
Int8Bound int8_bound_interval(int digits, int64_t lo, int64_t hi);
Int8Bound int8_bound_residues(uint64_t p);       // entries in [0, p), digits_for(p) digits
Int8Bound int8_bound_integers(int entry_bits);   // entries in [0, 2^entry_bits)
int64_t radix_top(int digits);                   // 127 (256^D - 1) / 255
size_t int8_workspace_bytes(int digits, int64_t m, int64_t n, int64_t k);
// planes made per call when A and/or B are resident (rounded up to 256 bytes)
size_t int8_planes_bytes(int digits, int64_t m, int64_t n, int64_t k, bool res_a, bool res_b);
// Multi-modular product of one integer pair (uint64 entries < 2^entry_bits)
// against up to kMaxPrimesCrt moduli, all from one digit GEMM; needs
// k <= int8_bound_integers(entry_bits).kblock.
constexpr int kMaxPrimesCrt = 64;
struct CrtLaunch {
  const uint64_t* A;
  const uint64_t* B;
  int64_t m, n, k, lda, ldb, ldc;
  int64_t kp;
  int nprimes;
  uint64_t p[kMaxPrimesCrt];
  double* C[kMaxPrimesCrt];
  int8_t* work;  // planes of A, then of B^T (digit_planes_bytes each)
};
int crt_digits(int entry_bits);  // fewest signed digits holding every value < 2^entry_bits
int launch_crt(int digits, const CrtLaunch& c, void* stream);

// Digit planes of one product into a.work, then the digit GEMM of up to
// kMaxBatch products with the same digit count (each with its own planes).
int launch_int8_digitize(int digits, const Int8Args& a, void* stream);
int launch_int8_gemm(int digits, const Int8Args* jobs, int njobs, void* stream);
// Digit planes and digit GEMM of up to 64 whole products (no resident
// planes, no split-K) of any digit counts: one launch each.
constexpr int kMaxMixedBatch = 64;
int launch_int8_batch(const Int8Args* jobs, const int* digits, int njobs, void* stream);

// Phase timer hooks (null tokens unless mmp_timers_enable(1)).  A launch
// passes timer_start(t) / timer_stop(t) as the start and stop events of
// hipExtLaunchKernelGGL, then hands the token back with timer_commit.
struct TimerTok {
  hipEvent_t e0, e1;
  const char* name;
};
TimerTok* timer_begin(const char* phase);
void timer_commit(TimerTok* t, int launch_status);
inline hipEvent_t timer_start(TimerTok* t) { return t ? t->e0 : nullptr; }
inline hipEvent_t timer_stop(TimerTok* t) { return t ? t->e1 : nullptr; }

// Up to kMaxBatch products of one kernel configuration in one launch; the
// job table travels in the kernel arguments (no device allocation, so a
// launch can be captured into a graph as is).
struct Fp64Batch {
  int njobs;
  int tile_start[kMaxBatch + 1];  // filled by the launcher
  Fp64Args job[kMaxBatch];
};
// Kernel class of a plan, 4 FE + 2 PAD + LAZY: FE = k-steps per in-loop
// reduction (1, 2 or 4), PAD = blocks leave zero slots in a stage
// (L < S <= 16), LAZY = correction-free in-loop reductions.  Jobs of one
// launch share it.
inline int fp64_class(int slots, int64_t kblock, bool lazy) {
  const int fe = slots == 4 ? 1 : slots == 8 ? 2 : 4;  // 4: a k-step counter, any S = 4j >= 12
  const int pad = (slots <= kBK && kblock < slots) ? 1 : 0;
  return 4 * fe + 2 * pad + (lazy ? 1 : 0);
}

// Launch the fused FP64-word kernel; returns a hipError_t value (0 = success).
int launch_fp64_words(int u, int v, int tile_id, const Fp64Batch& a, void* stream);
// Fill a row-major m x n matrix (leading dimension ld) with +0.0.
int launch_zero_fill(double* C, int64_t m, int64_t n, int64_t ld, void* stream);
// Scan for uint64 entries at or above 2^bits; sets *flag nonzero.
int launch_validate_bits(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, int bits, int* flag,
                         void* stream);
// out[r][c] = X[r][c] mod p as binary64 (integer reduction on the device).
int launch_reduce_mod(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, uint64_t p, double* out,
                      int64_t ldo, void* stream);

// Host helpers shared by the entry points (mmp_abi.cpp).
int hip_status(int err);
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes);
size_t span_bytes(int64_t rows, int64_t cols, int64_t ld);
// The FP64-word kernel addresses a stage's slabs with 32-bit byte offsets:
// BM rows of A and 16 k-rows of B must span less than 2^31 bytes.
bool fp64_ld_ok(const mmp_plan_t& pl, int64_t lda, int64_t ldb);
int check_product_args(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                       int64_t ldb, const double* C, int64_t ldc);
int acquire_workspace(size_t bytes, const mmp_opts* opts, void* stream, void** out, bool* owned);
int release_workspace(void* ptr, bool owned, void* stream);
int validate_product_entries(uint64_t p, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                             const double* B, int64_t ldb, void* stream);
int validate_integer_entries(int bits, int64_t m, int64_t n, int64_t k, const uint64_t* A, int64_t lda,
                             const uint64_t* B, int64_t ldb, void* stream);
Fp64Args make_fp64_args(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc);
Int8Args make_int8_args(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc, int8_t* work);

// Scan for entries outside [0, p) or non-integral; sets *flag (device int) nonzero.
int launch_validate(const double* X, int64_t rows, int64_t cols, int64_t ld, double p, int* flag,
                    void* stream);

}  // namespace mmp
