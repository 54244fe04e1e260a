// Small helper kernels (zero fill, entry validation) and the dispatcher over
// the per-(u, v) instantiations of the fused FP64-word kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mmp_internal.h"

namespace mmp {

#define MMP_DECL(U_, V_) int launch_fp64_words_##U_##_##V_(int tile_id, const Fp64Args& a, void* stream);
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

int launch_fp64_words(int u, int v, int tile_id, const Fp64Args& a, void* stream) {
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

#define MMP_DECL8(D_) int launch_int8_digits_##D_(const Int8Args& a, void* stream);
MMP_DECL8(1)
MMP_DECL8(2)
MMP_DECL8(3)
MMP_DECL8(4)
MMP_DECL8(5)
MMP_DECL8(6)
MMP_DECL8(7)
#undef MMP_DECL8

int launch_int8_digits(int digits, const Int8Args& a, void* stream) {
  switch (digits) {
    case 1: return launch_int8_digits_1(a, stream);
    case 2: return launch_int8_digits_2(a, stream);
    case 3: return launch_int8_digits_3(a, stream);
    case 4: return launch_int8_digits_4(a, stream);
    case 5: return launch_int8_digits_5(a, stream);
    case 6: return launch_int8_digits_6(a, stream);
    case 7: return launch_int8_digits_7(a, stream);
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

}  // namespace

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
