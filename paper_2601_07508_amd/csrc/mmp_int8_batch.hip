// Launchers of the batch-wide INT8 kernels (int8_digits_batch.h): the digit
// planes of up to kMaxMixedJobs products in one launch, then their digit
// GEMM in one persistent launch, whatever their digit counts.
#include <algorithm>
#include <atomic>
#include <cstring>

#include "int8_digits_batch.h"

namespace mmp {

int launch_int8_batch(const Int8Args* jobs, const int* digits, int njobs, void* stream) {
  using namespace i8d;
  if (njobs < 1 || njobs > kMaxMixedJobs) return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)stream;
  MixedBatch b;
  std::memset(&b, 0, sizeof(b));
  // The grid strides over the work items in table order, so the products
  // with the costliest tiles (digit products x k x tile width) go first and
  // the cheap tiles fill in at the end: every workgroup finishes close to
  // the others.
  int order[kMaxMixedJobs];
  for (int j = 0; j < njobs; j++) order[j] = j;
  auto tile_cost = [&](int j) { return (int64_t)digits[j] * digits[j] * jobs[j].kp * mixed_bn(digits[j]); };
  std::stable_sort(order, order + njobs, [&](int x, int y) { return tile_cost(x) > tile_cost(y); });
  int64_t dig = 0, tiles = 0;
  int n = 0;
  for (int jj = 0; jj < njobs; jj++) {
    const int j = order[jj];
    const Int8Args& g = jobs[j];
    const int D = digits[j];
    // whole products only: no resident planes, no split-K
    if (D < 1 || D > kMaxDigits || g.resident_a || g.resident_b || g.splits > 1) return (int)hipErrorInvalidValue;
    if (g.m <= 0 || g.n <= 0 || g.kp <= 0) continue;
    MixedJob& a = b.job[n++];
    a.A = g.A;
    a.B = g.B;
    a.Ad = g.work;
    a.Bd = g.work + digit_planes_bytes(D, g.m, g.kp);
    a.C = g.C;
    a.m = g.m;
    a.n = g.n;
    a.k = g.k;
    a.lda = g.lda;
    a.ldb = g.ldb;
    a.ldc = g.ldc;
    a.kp = g.kp;
    a.p = (double)g.p;
    a.q = g.q;
    int64_t top = 0;
    for (int i = 0; i < D; i++) top = top * 256 + 127;
    a.top = top;
    a.stages_per_block = g.kblock / kBK8;
    a.D = D;
    a.vec = ((uintptr_t)g.A % 16) == 0 && g.lda % 2 == 0;
    const int64_t gx = (g.kp + 127) / 128, gy = std::min<int64_t>((g.m + 15) / 16, 65535);
    a.gx = (int)gx;
    a.gy = (int)gy;
    a.dig_start = (int)dig;
    a.dig_cols = (int)(dig + gx * gy);
    dig += gx * gy + (g.kp / 64) * ((g.n + 63) / 64);
    a.tile_start = (int)tiles;
    tiles += ((g.m + 63) / 64) * ((g.n + mixed_bn(D) - 1) / mixed_bn(D));
    if (dig > 0x7fffffff || tiles > 0x7fffffff) return (int)hipErrorInvalidValue;
  }
  b.njobs = n;
  b.dig_total = (int)dig;
  b.tile_total = (int)tiles;
  if (n == 0) return 0;
  {
    TimerTok* t = timer_begin("int8_batch_digitize");
    hipExtLaunchKernelGGL(digitize_batch_kernel, dim3((unsigned)dig), dim3(256), 0, s, timer_start(t),
                          timer_stop(t), 0, b);
    const int e = (int)hipGetLastError();
    timer_commit(t, e);
    if (e) return e;
  }
  // the ring of the largest digit count, in dynamic LDS; a persistent grid of
  // as many workgroups as the device holds at once with that ring
  size_t lds = 0;  // the largest ring among the launch's digit counts
  for (int j = 0; j < n; j++) lds = std::max(lds, (size_t)mixed_ring_bytes(b.job[j].D));
  int dev = 0;
  if (int e = (int)hipGetDevice(&dev)) return e;
  static std::atomic<int> lds_ready[64];
  if (dev < 64 && !lds_ready[dev].load()) {
    int most = 0;
    for (int d = 1; d <= kMaxDigits; d++) most = std::max(most, (int)mixed_ring_bytes(d));
    if (int e = (int)hipFuncSetAttribute((const void*)int8_batch_gemm_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, most))
      return e;
    lds_ready[dev].store(1);
  }
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, int8_batch_gemm_kernel, 256, lds) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int64_t grid = std::min<int64_t>(tiles, (int64_t)cus * per_cu);
  TimerTok* t = timer_begin("int8_batch_gemm");
  hipExtLaunchKernelGGL(int8_batch_gemm_kernel, dim3((unsigned)grid), dim3(256), lds, s, timer_start(t),
                        timer_stop(t), 0, b);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

}  // namespace mmp
