// C-ABI entry points: argument checks, planning, launch, error mapping.
// Nothing here throws across the boundary; HIP failures become MMP_EHIP with
// the hipError_t kept per thread for mmp_last_hip_error().
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "mmp_internal.h"

namespace {

thread_local int g_last_hip_error = 0;

int hip_status(int err) {
  if (err == 0) return MMP_OK;
  g_last_hip_error = err;
  return err == (int)hipErrorOutOfMemory ? MMP_ENOMEM : MMP_EHIP;
}

// One device int per device for entry validation.
std::mutex g_flag_mu;
std::vector<int*> g_flags;

int* validation_flag(int dev) {
  std::lock_guard<std::mutex> lk(g_flag_mu);
  if ((int)g_flags.size() <= dev) g_flags.resize(dev + 1, nullptr);
  if (!g_flags[dev]) {
    int* f = nullptr;
    if (hipMalloc(&f, sizeof(int)) != hipSuccess) return nullptr;
    g_flags[dev] = f;
  }
  return g_flags[dev];
}

bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return abytes && bbytes && x < y + bbytes && y < x + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)(((rows - 1) * ld + cols) * (int64_t)sizeof(double));
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

// Stream-ordered workspace: the device's default memory pool, told to keep
// freed blocks cached so repeated calls do not return memory to the driver.
std::mutex g_pool_mu;
std::vector<char> g_pool_ready;

int prepare_pool(int dev) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pool_ready.size() <= dev) g_pool_ready.resize(dev + 1, 0);
  if (g_pool_ready[dev]) return 0;
  hipMemPool_t pool;
  if (hipError_t e = hipDeviceGetDefaultMemPool(&pool, dev)) return (int)e;
  uint64_t keep = UINT64_MAX;
  if (hipError_t e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep)) return (int)e;
  g_pool_ready[dev] = 1;
  return 0;
}

}  // namespace

extern "C" {

const char* mmp_strerror(int status) {
  switch (status) {
    case MMP_OK: return "success";
    case MMP_EINVAL: return "invalid argument";
    case MMP_EBOUND: return "no admissible block size for this modulus and word count";
    case MMP_ERANGE: return "matrix entry outside [0, p) or not an integer";
    case MMP_ENOMEM: return "out of memory";
    case MMP_EHIP: return "HIP runtime error";
    case MMP_EBUSY: return "admission rejected: server full";
    case MMP_ENOTFOUND: return "unknown ticket or handle";
    case MMP_ETIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

int mmp_last_hip_error(void) { return g_last_hip_error; }

int mmp_plan(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const mmp_opts* opts,
             mmp_plan_t* out) {
  try {
    return mmp::plan(p, u, v, m, n, k, opts, out);
  } catch (...) {
    return MMP_EINVAL;
  }
}

size_t mmp_footprint(const mmp_job* job, const mmp_plan_t* plan) {
  if (!job || job->m < 0 || job->n < 0 || job->k < 0) return 0;
  const size_t m = (size_t)job->m, n = (size_t)job->n, k = (size_t)job->k;
  size_t bytes = 8 * (m * k + k * n + m * n);
  if (plan) {
    if (plan->form == MMP_FORM_INT8_WORDS)
      bytes += (size_t)plan->digits_a * m * k + (size_t)plan->digits_b * k * n;
    else
      bytes += 8 * ((size_t)plan->u * m * k + (size_t)plan->v * k * n);
  }
  return bytes;
}

int mm_modp_async(const mmp_opts* opts, uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                  void* stream) {
  try {
    if (m < 0 || n < 0 || k < 0) return MMP_EINVAL;
    if (m > 0 && n > 0) {
      if (!C || ldc < n) return MMP_EINVAL;
      if (k > 0 && (!A || !B || lda < k || ldb < n)) return MMP_EINVAL;
      if (k > 0 && (ranges_overlap(C, span_bytes(m, n, ldc), A, span_bytes(m, k, lda)) ||
                    ranges_overlap(C, span_bytes(m, n, ldc), B, span_bytes(k, n, ldb))))
        return MMP_EINVAL;
    }
    mmp_plan_t pl;
    int st = mmp::plan(p, u, v, m, n, k, opts, &pl);
    if (st != MMP_OK) return st;
    if (m == 0 || n == 0) return MMP_OK;
    if (k == 0) return hip_status(mmp::launch_zero_fill(C, m, n, ldc, stream));

    if (opts && opts->validate_entries) {
      int dev = 0;
      if (int e = (int)hipGetDevice(&dev)) return hip_status(e);
      int* flag = validation_flag(dev);
      if (!flag) return MMP_ENOMEM;
      hipStream_t s = (hipStream_t)stream;
      if (int e = (int)hipMemsetAsync(flag, 0, sizeof(int), s)) return hip_status(e);
      if (int e = mmp::launch_validate(A, m, k, lda, (double)p, flag, stream)) return hip_status(e);
      if (int e = mmp::launch_validate(B, k, n, ldb, (double)p, flag, stream)) return hip_status(e);
      int host = 0;
      if (int e = (int)hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s))
        return hip_status(e);
      if (int e = (int)hipStreamSynchronize(s)) return hip_status(e);
      if (host) return MMP_ERANGE;
    }

    if (pl.form == MMP_FORM_INT8_WORDS) {
      hipStream_t s = (hipStream_t)stream;
      int dev = 0;
      if (int e = (int)hipGetDevice(&dev)) return hip_status(e);
      if (int e = prepare_pool(dev)) return hip_status(e);
      void* work = nullptr;
      if (int e = (int)hipMallocAsync(&work, pl.workspace_bytes, s)) return hip_status(e);
      mmp::Int8Args g;
      std::memset(&g, 0, sizeof(g));
      g.A = A;
      g.B = B;
      g.C = C;
      g.m = m;
      g.n = n;
      g.k = k;
      g.lda = lda;
      g.ldb = ldb;
      g.ldc = ldc;
      g.kp = (k + 63) / 64 * 64;
      g.p = p;
      g.q = pl.q;
      g.kblock = pl.kblock_int8;
      g.work = (int8_t*)work;
      int e = mmp::launch_int8_digits(pl.digits_a, g, stream);
      int e2 = (int)hipFreeAsync(work, s);
      return hip_status(e ? e : e2);
    }

    mmp::Fp64Args a;
    std::memset(&a, 0, sizeof(a));
    a.A = A;
    a.B = B;
    a.C = C;
    a.m = m;
    a.n = n;
    a.k = k;
    a.lda = lda;
    a.ldb = ldb;
    a.ldc = ldc;
    a.p = (double)p;
    a.q = pl.q;
    a.alpha = (double)pl.alpha;
    a.beta = (double)pl.beta;
    a.ainv = (pl.u > 1 && is_pow2(pl.alpha)) ? 1.0 / (double)pl.alpha : 0.0;
    a.binv = (pl.v > 1 && is_pow2(pl.beta)) ? 1.0 / (double)pl.beta : 0.0;
    a.L = (int)pl.kblock;
    a.S = pl.slots;
    a.KR = (pl.slots <= mmp::kBK) ? (mmp::kBK / pl.slots) * (int)pl.kblock : mmp::kBK;
    a.stages_per_block = pl.slots >= mmp::kBK ? pl.slots / mmp::kBK : 1;
    a.lazy = pl.lazy;
    return hip_status(mmp::launch_fp64_words(pl.u, pl.v, pl.tile, a, stream));
  } catch (...) {
    return MMP_EINVAL;
  }
}

int mm_modp(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k, const double* A,
            const double* B, double* C) {
  int st = mm_modp_async(nullptr, p, u, v, m, n, k, A, k, B, n, C, n, nullptr);
  if (st != MMP_OK || m == 0 || n == 0) return st;  // empty products enqueue nothing
  return hip_status((int)hipStreamSynchronize(nullptr));
}

}  // extern "C"
