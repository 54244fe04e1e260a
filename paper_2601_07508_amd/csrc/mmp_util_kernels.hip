// Small helper kernels (zero fill, entry validation) and the dispatcher over
// the per-(u, v) instantiations of the fused FP64-word kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mmp_internal.h"

namespace mmp {

#define MMP_DECL(U_, V_) int launch_fp64_words_##U_##_##V_(int tile_id, const Fp64Batch& a, void* stream);
MMP_DECL(1, 1)
MMP_DECL(1, 2)
MMP_DECL(2, 1)
MMP_DECL(1, 3)
MMP_DECL(3, 1)
MMP_DECL(2, 2)
MMP_DECL(1, 4)
MMP_DECL(4, 1)
MMP_DECL(2, 3)
MMP_DECL(3, 2)
MMP_DECL(2, 4)
MMP_DECL(4, 2)
#undef MMP_DECL

int launch_fp64_words(int u, int v, int tile_id, const Fp64Batch& a, void* stream) {
#define MMP_UV(U_, V_) \
  if (u == U_ && v == V_) return launch_fp64_words_##U_##_##V_(tile_id, a, stream);
  MMP_UV(1, 1)
  MMP_UV(1, 2)
  MMP_UV(2, 1)
  MMP_UV(1, 3)
  MMP_UV(3, 1)
  MMP_UV(2, 2)
  MMP_UV(1, 4)
  MMP_UV(4, 1)
  MMP_UV(2, 3)
  MMP_UV(3, 2)
  MMP_UV(2, 4)
  MMP_UV(4, 2)
#undef MMP_UV
  return (int)hipErrorInvalidValue;
}

#define MMP_DECL8(D_)                                                                               \
  int launch_int8_digitize_##D_(const Int8Args& a, void* stream);                                   \
  int launch_int8_gemm_##D_(const Int8Args* jobs, int njobs, void* stream);                         \
  int launch_int8_digitize_side_##D_(int side, const double* X, int64_t rows, int64_t cols, int64_t ld, \
                                     int64_t kp, uint64_t p, int8_t* out, void* stream);
MMP_DECL8(1)
MMP_DECL8(2)
MMP_DECL8(3)
MMP_DECL8(4)
MMP_DECL8(5)
MMP_DECL8(6)
MMP_DECL8(7)
#undef MMP_DECL8

#define MMP_DECLC(D_) int launch_crt_##D_(const CrtLaunch& c, void* stream);
MMP_DECLC(1)
MMP_DECLC(2)
MMP_DECLC(3)
MMP_DECLC(4)
MMP_DECLC(5)
MMP_DECLC(6)
MMP_DECLC(7)
MMP_DECLC(8)
#undef MMP_DECLC

int launch_crt(int digits, const CrtLaunch& c, void* stream) {
  switch (digits) {
    case 1: return launch_crt_1(c, stream);
    case 2: return launch_crt_2(c, stream);
    case 3: return launch_crt_3(c, stream);
    case 4: return launch_crt_4(c, stream);
    case 5: return launch_crt_5(c, stream);
    case 6: return launch_crt_6(c, stream);
    case 7: return launch_crt_7(c, stream);
    case 8: return launch_crt_8(c, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_int8_digitize(int digits, const Int8Args& a, void* stream) {
  switch (digits) {
    case 1: return launch_int8_digitize_1(a, stream);
    case 2: return launch_int8_digitize_2(a, stream);
    case 3: return launch_int8_digitize_3(a, stream);
    case 4: return launch_int8_digitize_4(a, stream);
    case 5: return launch_int8_digitize_5(a, stream);
    case 6: return launch_int8_digitize_6(a, stream);
    case 7: return launch_int8_digitize_7(a, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_int8_digitize_side(int digits, int side, const double* X, int64_t rows, int64_t cols, int64_t ld,
                              int64_t kp, uint64_t p, int8_t* out, void* stream) {
#define MMP_SIDE(D_) \
  case D_: return launch_int8_digitize_side_##D_(side, X, rows, cols, ld, kp, p, out, stream);
  switch (digits) {
    MMP_SIDE(1)
    MMP_SIDE(2)
    MMP_SIDE(3)
    MMP_SIDE(4)
    MMP_SIDE(5)
    MMP_SIDE(6)
    MMP_SIDE(7)
    default: return (int)hipErrorInvalidValue;
  }
#undef MMP_SIDE
}

int launch_int8_gemm(int digits, const Int8Args* jobs, int njobs, void* stream) {
  switch (digits) {
    case 1: return launch_int8_gemm_1(jobs, njobs, stream);
    case 2: return launch_int8_gemm_2(jobs, njobs, stream);
    case 3: return launch_int8_gemm_3(jobs, njobs, stream);
    case 4: return launch_int8_gemm_4(jobs, njobs, stream);
    case 5: return launch_int8_gemm_5(jobs, njobs, stream);
    case 6: return launch_int8_gemm_6(jobs, njobs, stream);
    case 7: return launch_int8_gemm_7(jobs, njobs, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

namespace {

__global__ void zero_fill_kernel(double* C, int64_t m, int64_t n, int64_t ld) {
  const int64_t total = m * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, c = i - (i / n) * n;
    C[r * ld + c] = 0.0;
  }
}

__global__ void validate_kernel(const double* X, int64_t rows, int64_t cols, int64_t ld, double p,
                                int* flag) {
  const int64_t total = rows * cols;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - (i / cols) * cols;
    const double x = X[r * ld + c];
    if (!(x >= 0.0 && x < p && x == floor(x))) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void validate_bits_kernel(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, int bits,
                                     int* flag) {
  const int64_t total = rows * cols;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - (i / cols) * cols;
    if ((X[r * ld + c] >> bits) != 0) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void reduce_mod_kernel(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, uint64_t p,
                                  double* out, int64_t ldo) {
  const int64_t total = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i - (i / cols) * cols;
    out[r * ldo + c] = (double)(X[r * ld + c] % p);
  }
}

__global__ void splitk_reduce_kernel(const double* P, int splits, int64_t m, int64_t n, double p, double* C,
                                     int64_t ldc) {
  const int64_t total = m * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < splits; t++) {  // residues in [0, p): exact modular adds
      s += P[t * total + i];
      s = (s >= p) ? s - p : s;
    }
    const int64_t r = i / n, c = i - (i / n) * n;
    C[r * ldc + c] = s + 0.0;
  }
}

__global__ void fill_mod_kernel(double* X, int64_t count, uint64_t p, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;  // SplitMix64 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    X[i] = (double)(z % p);
  }
}

}  // namespace

int launch_splitk_reduce(const double* partial, int splits, int64_t m, int64_t n, double p, double* C, int64_t ldc,
                         void* stream) {
  if (m <= 0 || n <= 0) return 0;
  const int64_t total = m * n;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  TimerTok* t = timer_begin("splitk_reduce");
  hipExtLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                        timer_start(t), timer_stop(t), 0, partial, splits, m, n, p, C, ldc);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

int choose_splits(int64_t tiles, int64_t stages, int64_t min_stages_per_split) {
  // The FP64-word kernel.  Output tiles that cannot fill 256 CUs twice get k-ranges: enough for four
  // rounds of 512 workgroups, so that the last, partly filled round costs
  // little (with one or two rounds a 171-tile product spent a third of its
  // time in a round a third full), each split a sizeable k-range; a power
  // of two, so that from 8 on every XCD of the round-robin dispatch owns
  // whole k-ranges (the kernels put the k-range in the low bits of the
  // workgroup id)
  if (tiles <= 0 || tiles >= 512 || stages < 2 * min_stages_per_split) return 1;
  const int64_t want = (4 * 512 + tiles - 1) / tiles;
  const int64_t cap = std::min<int64_t>(stages / min_stages_per_split, 64);
  int64_t s = 1;
  while (s < want && 2 * s <= cap) s *= 2;
  return (int)s;
}

int choose_splits_fill(int64_t tiles, int64_t stages, int64_t min_stages_per_split) {
  // The digit GEMM: the fewest k-ranges (a power of two) that fill one round
  // of 512 workgroups, doubled while the last round is less than 90% full.
  // More k-ranges than that cost time here: each XCD then holds several
  // k-ranges' digit slabs at once in its L2 (512 x 512 x 131072 at 23 bits:
  // 0.395 ms at 8 k-ranges, 0.496 ms at 32).
  if (tiles <= 0 || tiles >= 512 || stages < 2 * min_stages_per_split) return 1;
  const int64_t cap = std::min<int64_t>(stages / min_stages_per_split, 64);
  int64_t s = 1;
  while (tiles * s < 512 && 2 * s <= cap) s *= 2;
  auto fill = [&](int64_t x) {
    const int64_t w = tiles * x, rounds = (w + 511) / 512;
    return (double)w / (double)(512 * rounds);
  };
  while (fill(s) < 0.9 && 2 * s <= cap) s *= 2;
  return (int)s;
}

int launch_fill_mod(double* X, int64_t count, uint64_t p, uint64_t seed, void* stream) {
  if (count <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_mod_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, X, count, p, seed);
  return (int)hipGetLastError();
}

int launch_validate_bits(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, int bits, int* flag,
                         void* stream) {
  if (rows <= 0 || cols <= 0) return 0;
  const int64_t total = rows * cols;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(validate_bits_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, X, rows,
                     cols, ld, bits, flag);
  return (int)hipGetLastError();
}

int launch_reduce_mod(const uint64_t* X, int64_t rows, int64_t cols, int64_t ld, uint64_t p, double* out,
                      int64_t ldo, void* stream) {
  if (rows <= 0 || cols <= 0) return 0;
  const int64_t total = rows * cols;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(reduce_mod_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, X, rows,
                     cols, ld, p, out, ldo);
  return (int)hipGetLastError();
}

int launch_zero_fill(double* C, int64_t m, int64_t n, int64_t ld, void* stream) {
  if (m <= 0 || n <= 0) return 0;
  const int64_t total = m * n;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, C, m,
                     n, ld);
  return (int)hipGetLastError();
}

int launch_validate(const double* X, int64_t rows, int64_t cols, int64_t ld, double p, int* flag,
                    void* stream) {
  if (rows <= 0 || cols <= 0) return 0;
  const int64_t total = rows * cols;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, X, rows,
                     cols, ld, p, flag);
  return (int)hipGetLastError();
}
}  // namespace mmp
