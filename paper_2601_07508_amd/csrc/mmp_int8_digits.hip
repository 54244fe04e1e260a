// One digit count D of the INT8-digit form, selected at build time by MMP_D:
// the digitizing passes of one product and the digit GEMM of a batch.
#include <atomic>

#include "int8_crt_kernel.h"
#include "int8_digits_kernel.h"
#include "int8_digits_persistent.h"

#if !defined(MMP_D)
#error "build with -DMMP_D=<digits>"
#endif

#define MMP_CAT2(a, b) a##b
#define MMP_CAT(a, b) MMP_CAT2(a, b)

namespace mmp {

namespace {
// Row digitizing launch: x over 128-column chunks, y over 16-row groups
// (strided beyond 65535); the vector form when every row starts 16-byte
// aligned.
template <int D, class In, class T>
hipError_t launch_digitize_rows(const In& in, const T* X, int64_t rows, int64_t cols, int64_t ld, int64_t kp,
                                int8_t* out, hipStream_t s, TimerTok* t) {
  if (rows <= 0 || kp <= 0) return hipSuccess;
  if ((kp + 127) / 128 > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((kp + 127) / 128), (unsigned)std::min<int64_t>((rows + 15) / 16, 65535));
  if (((uintptr_t)X % 16) == 0 && ld % 2 == 0)
    hipExtLaunchKernelGGL((i8d::digitize_rows_kernel<D, In, true>), grid, dim3(256), 0, s, timer_start(t),
                          timer_stop(t), 0, in, rows, cols, ld, kp, out);
  else
    hipExtLaunchKernelGGL((i8d::digitize_rows_kernel<D, In, false>), grid, dim3(256), 0, s, timer_start(t),
                          timer_stop(t), 0, in, rows, cols, ld, kp, out);
  return hipGetLastError();
}
}  // namespace

#if MMP_D <= 7  // residues of p < 2^52 need at most 7 digits

// side 0: X is A (rows x cols = m x k) -> D planes of m x kp;
// side 1: X is B (rows x cols = k x n) -> D transposed planes of n x kp.
int MMP_CAT(launch_int8_digitize_side_, MMP_D)(int side, const double* X, int64_t rows, int64_t cols, int64_t ld,
                                               int64_t kp, uint64_t p, int8_t* out, void* stream) {
  using namespace i8d;
  constexpr int D = MMP_D;
  hipStream_t s = (hipStream_t)stream;
  // largest value D signed base-256 digits reach: 127 (256^D - 1) / 255
  int64_t top = 0;
  for (int i = 0; i < D; i++) top = top * 256 + 127;
  const ResidueIn in{X, (int64_t)p, top};
  if (side == 0) {
    TimerTok* t = timer_begin("int8_digitize_a");
    const hipError_t e = launch_digitize_rows<D>(in, X, rows, cols, ld, kp, out, s, t);
    timer_commit(t, (int)e);
    return (int)e;
  }
  const int64_t tiles = (kp / 64) * ((cols + 63) / 64);
  if (tiles > 0x7fffffff) return (int)hipErrorInvalidValue;
  TimerTok* t = timer_begin("int8_digitize_b");
  hipExtLaunchKernelGGL((digitize_cols_kernel<D, ResidueIn>), dim3((unsigned)tiles), dim3(256), 0, s,
                        timer_start(t), timer_stop(t), 0, in, rows, cols, ld, kp, out);
  const hipError_t e = hipGetLastError();
  timer_commit(t, (int)e);
  return (int)e;
}

int MMP_CAT(launch_int8_digitize_, MMP_D)(const Int8Args& g, void* stream) {
  using namespace i8d;
  constexpr int D = MMP_D;
  // planes made here: A's (unless resident), then B's (unless resident)
  int8_t* Ad = g.work;
  int8_t* Bd = g.work + (g.resident_a ? (size_t)0 : digit_planes_bytes(D, g.m, g.kp));
  if (!g.resident_a && !g.resident_b && g.m > 0 && g.n > 0 && g.kp > 0) {
    // both operands: one launch (A's row part, then B's column tiles)
    int64_t top = 0;
    for (int i = 0; i < D; i++) top = top * 256 + 127;
    const ResidueIn ia{g.A, (int64_t)g.p, top}, ib{g.B, (int64_t)g.p, top};
    const int64_t gx = (g.kp + 127) / 128, gy = std::min<int64_t>((g.m + 15) / 16, 65535);
    const int64_t total = gx * gy + (g.kp / 64) * ((g.n + 63) / 64);
    if (total > 0x7fffffff) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    TimerTok* t = timer_begin("int8_digitize");
    if (((uintptr_t)g.A % 16) == 0 && g.lda % 2 == 0)
      hipExtLaunchKernelGGL((digitize_pair_kernel<D, ResidueIn, true>), dim3((unsigned)total), dim3(256), 0, s,
                            timer_start(t), timer_stop(t), 0, ia, g.m, g.k, g.lda, ib, g.n, g.ldb, g.kp, Ad, Bd, gx,
                            gy);
    else
      hipExtLaunchKernelGGL((digitize_pair_kernel<D, ResidueIn, false>), dim3((unsigned)total), dim3(256), 0, s,
                            timer_start(t), timer_stop(t), 0, ia, g.m, g.k, g.lda, ib, g.n, g.ldb, g.kp, Ad, Bd, gx,
                            gy);
    const hipError_t e = hipGetLastError();
    timer_commit(t, (int)e);
    return (int)e;
  }
  if (!g.resident_a)
    if (int e = MMP_CAT(launch_int8_digitize_side_, MMP_D)(0, g.A, g.m, g.k, g.lda, g.kp, g.p, Ad, stream)) return e;
  if (!g.resident_b)
    if (int e = MMP_CAT(launch_int8_digitize_side_, MMP_D)(1, g.B, g.k, g.n, g.ldb, g.kp, g.p, Bd, stream)) return e;
  return 0;
}

namespace {
i8d::GemmArgs gemm_args(const Int8Args& g) {
  using namespace i8d;
  GemmArgs a;
  a.Ad = g.resident_a ? g.resident_a : g.work;
  a.Bd = g.resident_b ? g.resident_b : g.work + (g.resident_a ? (size_t)0 : digit_planes_bytes(MMP_D, g.m, g.kp));
  a.C = g.C;
  a.m = g.m;
  a.n = g.n;
  a.kp = g.kp;
  a.ldc = g.ldc;
  a.p = (double)g.p;
  a.q = g.q;
  a.stages_per_block = g.kblock / kBK8;
  a.splits = g.splits < 1 ? 1 : g.splits;
  a.partial = g.partial;
  return a;
}

template <bool NARROW>
int launch_gemm(const Int8Args* jobs, int njobs, hipStream_t s) {
  using namespace i8d;
  constexpr int D = MMP_D;
  using S = I8Shape<D, NARROW>;
  constexpr int BM = S::BM, BN = S::BN;
  GemmBatch b;
  b.njobs = njobs;
  int64_t total = 0;
  for (int j = 0; j < njobs; j++) {
    const Int8Args& g = jobs[j];
    GemmArgs& a = b.job[j];
    a = gemm_args(g);
    b.tile_start[j] = (int)total;
    total += ((g.m + BM - 1) / BM) * ((g.n + BN - 1) / BN) * a.splits;
    if (total > 0x7fffffff) return (int)hipErrorInvalidValue;
  }
  b.tile_start[njobs] = (int)total;
  if (total <= 0) return 0;
  TimerTok* t = timer_begin("int8_gemm");
  hipExtLaunchKernelGGL((int8_digits_gemm_kernel<D, NARROW>), dim3((unsigned)total), dim3(S::THREADS), 0, s,
                        timer_start(t), timer_stop(t), 0, b);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

// Workgroups of the persistent kernel the current device holds at once:
// compute units x resident workgroups per unit (registers and LDS decide;
// cached per device).
template <int D>
int64_t persistent_slots() {
  static std::atomic<int64_t> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  if (dev < 64) {
    const int64_t c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, i8d::int8_digits_gemm_persistent_kernel<D>,
                                                   i8d::I8Shape<D, false>::THREADS, 0) != hipSuccess ||
      per_cu <= 0)
    per_cu = i8d::I8Shape<D, false>::GROUPS_PER_CU;
  const int64_t slots = (int64_t)cus * per_cu;
  if (dev < 64) cache[dev].store(slots, std::memory_order_relaxed);
  return slots;
}

// One product of 64 x 64 tiles whose tiles are short (at most
// kPersistentMaxStages k-stages, whole k per tile, within one int32 block),
// at least twice as many as the device holds workgroups, and each operand's
// planes below 4 GB in all (the kernel keeps 32-bit copy offsets from an
// operand's first plane): the persistent kernel, one workgroup per resident
// slot.
constexpr int64_t kPersistentMaxStages = 16;
int launch_persistent_if_short(const Int8Args& g, hipStream_t s, bool* launched) {
  using namespace i8d;
  constexpr int D = MMP_D;
  using S = I8Shape<D, false>;
  *launched = false;
  if (g.splits > 1 || g.kp <= 0 || g.kp / kBK8 > kPersistentMaxStages || g.kp > g.kblock) return 0;
  if (digit_planes_bytes(D, std::max(g.m, g.n), g.kp) >= ((size_t)1 << 32)) return 0;
  const int64_t tiles = ((g.m + S::BM - 1) / S::BM) * ((g.n + S::BN - 1) / S::BN);
  const int64_t slots = persistent_slots<D>();
  if (tiles < 2 * slots || tiles > 0x7fffffff) return 0;
  const GemmArgs a = gemm_args(g);
  *launched = true;
  TimerTok* t = timer_begin("int8_gemm_persistent");
  hipExtLaunchKernelGGL((int8_digits_gemm_persistent_kernel<D>), dim3((unsigned)slots), dim3(S::THREADS), 0, s,
                        timer_start(t), timer_stop(t), 0, a);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}
}  // namespace

// 64 x 32 tiles when every product of the launch has n <= 32, else 64 x 64
// (a lone product of many short tiles on the persistent kernel).
int MMP_CAT(launch_int8_gemm_, MMP_D)(const Int8Args* jobs, int njobs, void* stream) {
  if (njobs < 1 || njobs > kMaxBatch) return (int)hipErrorInvalidValue;
  bool narrow = true;
  for (int j = 0; j < njobs; j++) narrow = narrow && jobs[j].n <= 32;
  if (narrow) return launch_gemm<true>(jobs, njobs, (hipStream_t)stream);
  if (njobs == 1) {
    bool launched = false;
    const int e = launch_persistent_if_short(jobs[0], (hipStream_t)stream, &launched);
    if (launched) return e;
  }
  return launch_gemm<false>(jobs, njobs, (hipStream_t)stream);
}

#endif

int MMP_CAT(launch_crt_, MMP_D)(const CrtLaunch& c, void* stream) {
  using namespace i8d;
  constexpr int D = MMP_D;
  constexpr int BM = I8Shape<D>::BM, BN = I8Shape<D>::BN;
  static_assert(kMaxPrimes == kMaxPrimesCrt, "prime table sizes");
  hipStream_t s = (hipStream_t)stream;
  if (c.nprimes < 1 || c.nprimes > kMaxPrimes) return (int)hipErrorInvalidValue;
  const int64_t kp = c.kp;
  int8_t* Ad = c.work;
  int8_t* Bd = c.work + digit_planes_bytes(D, c.m, kp);
  {
    const IntegerIn in{c.A};
    TimerTok* t = timer_begin("crt_digitize_a");
    const hipError_t e = launch_digitize_rows<D>(in, c.A, c.m, c.k, c.lda, kp, Ad, s, t);
    timer_commit(t, (int)e);
    if (e) return (int)e;
  }
  {
    const IntegerIn in{c.B};
    const int64_t tiles = (kp / 64) * ((c.n + 63) / 64);
    if (tiles > 0x7fffffff) return (int)hipErrorInvalidValue;
    TimerTok* t = timer_begin("crt_digitize_b");
    hipExtLaunchKernelGGL((digitize_cols_kernel<D, IntegerIn>), dim3((unsigned)tiles), dim3(256), 0, s,
                          timer_start(t), timer_stop(t), 0, in, c.k, c.n, c.ldb, kp, Bd);
    const hipError_t e = hipGetLastError();
    timer_commit(t, (int)e);
    if (e) return (int)e;
  }
  CrtArgs a;
  a.Ad = Ad;
  a.Bd = Bd;
  a.m = c.m;
  a.n = c.n;
  a.kp = kp;
  a.ldc = c.ldc;
  a.nprimes = c.nprimes;
  // fold_direct's condition: Gmax = 65793 kp D 2^14 <= (2^27 - 2) p for
  // every modulus (exact in 128-bit integers)
  const unsigned __int128 gmax = (unsigned __int128)65793 * (uint64_t)kp * (uint64_t)D * 16384u;
  a.direct = 1;
  for (int i = 0; i < c.nprimes; i++) {
    a.p[i] = (double)c.p[i];
    a.q[i] = 1.0 / (double)c.p[i];
    a.C[i] = c.C[i];
    if (gmax > (unsigned __int128)((1ull << 27) - 2) * c.p[i]) a.direct = 0;
  }
  const int64_t nb = ((c.m + BM - 1) / BM) * ((c.n + BN - 1) / BN);
  if (nb <= 0) return 0;
  if (nb > 0x7fffffff) return (int)hipErrorInvalidValue;
  TimerTok* t = timer_begin("crt_gemm");
  hipExtLaunchKernelGGL((crt_gemm_kernel<D>), dim3((unsigned)nb), dim3(I8Shape<D>::THREADS), 0, s,
                        timer_start(t), timer_stop(t), 0, a);
  const int e = (int)hipGetLastError();
  timer_commit(t, e);
  return e;
}

}  // namespace mmp
