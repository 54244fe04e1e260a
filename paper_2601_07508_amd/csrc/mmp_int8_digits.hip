// One digit count D of the INT8-digit form, selected at build time by MMP_D.
#include "int8_digits_kernel.h"

#if !defined(MMP_D)
#error "build with -DMMP_D=<digits>"
#endif

#define MMP_CAT2(a, b) a##b
#define MMP_CAT(a, b) MMP_CAT2(a, b)

namespace mmp {

int MMP_CAT(launch_int8_digits_, MMP_D)(const Int8Args& g, void* stream) {
  using namespace i8d;
  constexpr int D = MMP_D;
  hipStream_t s = (hipStream_t)stream;
  // largest value D signed base-256 digits reach: 127 (256^D - 1) / 255
  int64_t top = 0;
  for (int i = 0; i < D; i++) top = top * 256 + 127;
  const int64_t kp = g.kp;
  int8_t* Ad = g.work;
  int8_t* Bd = g.work + (size_t)D * g.m * kp;
  {
    const int64_t total = g.m * (kp / 4);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL((digitize_rows_kernel<D>), dim3((unsigned)blocks), dim3(256), 0, s, g.A, g.m, g.k,
                       g.lda, kp, (int64_t)g.p, top, Ad);
    if (hipError_t e = hipGetLastError()) return (int)e;
  }
  {
    const int64_t tiles = (kp / 64) * ((g.n + 63) / 64);
    if (tiles > 0x7fffffff) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((digitize_cols_kernel<D>), dim3((unsigned)tiles), dim3(256), 0, s, g.B, g.k, g.n,
                       g.ldb, kp, (int64_t)g.p, top, Bd);
    if (hipError_t e = hipGetLastError()) return (int)e;
  }
  constexpr int TM = I8Tile<D>::tm, TN = I8Tile<D>::tn;
  constexpr int BM = 32 * TM, BN = 32 * TN;
  const int64_t nb = ((g.m + BM - 1) / BM) * ((g.n + BN - 1) / BN);
  if (nb > 0x7fffffff) return (int)hipErrorInvalidValue;
  GemmArgs a;
  a.Ad = Ad;
  a.Bd = Bd;
  a.C = g.C;
  a.m = g.m;
  a.n = g.n;
  a.kp = kp;
  a.ldc = g.ldc;
  a.p = (double)g.p;
  a.q = g.q;
  a.stages_per_block = g.kblock / kBK8;
  hipLaunchKernelGGL((int8_digits_gemm_kernel<D, TM, TN>), dim3((unsigned)nb), dim3(kThreads), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mmp
