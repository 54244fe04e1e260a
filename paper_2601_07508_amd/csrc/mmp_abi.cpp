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
}  // namespace

namespace mmp {

int hip_status(int err) {
  if (err == 0) return MMP_OK;
  g_last_hip_error = err;
  return err == (int)hipErrorOutOfMemory ? MMP_ENOMEM : MMP_EHIP;
}

}  // namespace mmp

namespace {
using mmp::hip_status;

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

}  // namespace

namespace mmp {

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

bool fp64_ld_ok(const mmp_plan_t& pl, int64_t lda, int64_t ldb) {
  if (pl.form != MMP_FORM_FP64_WORDS) return true;
  const int64_t lim = (int64_t)1 << 31;
  return ((int64_t)(pl.bm - 1) * lda + kBK) * 8 < lim && ((int64_t)kBK * ldb + pl.bn) * 8 < lim;
}

int check_product_args(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda, const double* B,
                       int64_t ldb, const double* C, int64_t ldc) {
  if (m < 0 || n < 0 || k < 0) return MMP_EINVAL;
  if (m > 0 && n > 0) {
    if (!C || ldc < n) return MMP_EINVAL;
    if (k > 0 && (!A || !B || lda < k || ldb < n)) return MMP_EINVAL;
    if (k > 0 && (ranges_overlap(C, span_bytes(m, n, ldc), A, span_bytes(m, k, lda)) ||
                  ranges_overlap(C, span_bytes(m, n, ldc), B, span_bytes(k, n, ldb))))
      return MMP_EINVAL;
  }
  return MMP_OK;
}

// Prepared planes describe the operand a product reads: same side, modulus,
// shape and digit count.
bool operand_fits(const mmp_operand_t& o, int side, uint64_t p, int64_t rows, int64_t cols, int digits) {
  const int64_t inner = side == 0 ? cols : rows;
  return o.planes && o.side == side && o.p == p && o.rows == rows && o.cols == cols && o.digits == digits &&
         o.kp == (inner + 63) / 64 * 64;
}

// Stream-ordered workspace: the device's default memory pool, told to keep
// freed blocks cached so repeated calls do not return memory to the driver.
static std::mutex g_pool_mu;
static std::vector<char> g_pool_ready;

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

int acquire_workspace(size_t bytes, const mmp_opts* opts, void* stream, void** out, bool* owned) {
  *out = nullptr;
  *owned = false;
  if (bytes == 0) return MMP_OK;
  if (opts && opts->workspace) {
    if (opts->workspace_bytes < bytes) return MMP_EINVAL;
    *out = opts->workspace;
    return MMP_OK;
  }
  int dev = 0;
  if (int e = (int)hipGetDevice(&dev)) return hip_status(e);
  if (int e = prepare_pool(dev)) return hip_status(e);
  if (int e = (int)hipMallocAsync(out, bytes, (hipStream_t)stream)) return hip_status(e);
  *owned = true;
  return MMP_OK;
}

int release_workspace(void* ptr, bool owned, void* stream) {
  if (!owned || !ptr) return MMP_OK;
  return hip_status((int)hipFreeAsync(ptr, (hipStream_t)stream));
}

int validate_product_entries(uint64_t p, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                             const double* B, int64_t ldb, void* stream) {
  int dev = 0;
  if (int e = (int)hipGetDevice(&dev)) return hip_status(e);
  int* flag = validation_flag(dev);
  if (!flag) return MMP_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (int e = (int)hipMemsetAsync(flag, 0, sizeof(int), s)) return hip_status(e);
  if (int e = launch_validate(A, m, k, lda, (double)p, flag, stream)) return hip_status(e);
  if (int e = launch_validate(B, k, n, ldb, (double)p, flag, stream)) return hip_status(e);
  int host = 0;
  if (int e = (int)hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s)) return hip_status(e);
  if (int e = (int)hipStreamSynchronize(s)) return hip_status(e);
  return host ? MMP_ERANGE : MMP_OK;
}

int validate_integer_entries(int bits, int64_t m, int64_t n, int64_t k, const uint64_t* A, int64_t lda,
                             const uint64_t* B, int64_t ldb, void* stream) {
  int dev = 0;
  if (int e = (int)hipGetDevice(&dev)) return hip_status(e);
  int* flag = validation_flag(dev);
  if (!flag) return MMP_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (int e = (int)hipMemsetAsync(flag, 0, sizeof(int), s)) return hip_status(e);
  if (int e = launch_validate_bits(A, m, k, lda, bits, flag, stream)) return hip_status(e);
  if (int e = launch_validate_bits(B, k, n, ldb, bits, flag, stream)) return hip_status(e);
  int host = 0;
  if (int e = (int)hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, s)) return hip_status(e);
  if (int e = (int)hipStreamSynchronize(s)) return hip_status(e);
  return host ? MMP_ERANGE : MMP_OK;
}

Fp64Args make_fp64_args(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc) {
  Fp64Args a;
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
  a.p = (double)pl.p;
  a.q = pl.q;
  a.alpha = (double)pl.alpha;
  a.beta = (double)pl.beta;
  a.ainv = 1.0 / (double)pl.alpha;
  a.binv = 1.0 / (double)pl.beta;
  a.afix = (pl.u > 1 && !is_pow2(pl.alpha)) ? 1 : 0;
  a.bfix = (pl.v > 1 && !is_pow2(pl.beta)) ? 1 : 0;
  a.L = (int)pl.kblock;
  a.S = pl.slots;
  // real k-terms per 16-slot stage: fewer only when blocks leave zero slots
  a.KR = (pl.slots <= kBK && pl.kblock < pl.slots) ? (kBK / pl.slots) * (int)pl.kblock : kBK;
  a.ksteps_per_block = pl.slots / 4;
  a.lazy = pl.lazy;
  a.splits = 1;
  if (pl.biased) {  // biased reduction: the extended bound, or a paper block that needs the signed range
    const uint64_t K = (kTwoT / pl.p) - 1;  // K p <= 2^t - p
    a.bias = (double)K;
    a.acc_init = -(double)(K * pl.p);
  }
  if (pl.centered) {  // quotient rounded to nearest: c = floor(x q + 1/2)
    a.centered = 1;
    a.bias = 0.5;
    a.acc_init = 0.0;
    a.lazy = 1;
  }
  return a;
}

Int8Args make_int8_args(const mmp_plan_t& pl, int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                        const double* B, int64_t ldb, double* C, int64_t ldc, int8_t* work) {
  Int8Args g;
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
  g.p = pl.p;
  g.q = pl.q;
  g.kblock = pl.kblock_int8;
  g.work = work;
  g.splits = 1;
  return g;
}

}  // namespace mmp

namespace {
using namespace mmp;

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

static void copy_bound(const mmp::Int8Bound& b, mmp_int8_bound_t* out) {
  out->digits = b.digits;
  out->weight_max = b.weight_max;
  out->weight_min = b.weight_min;
  out->lo = b.lo;
  out->hi = b.hi;
  out->term_max = b.term_max;
  out->term_min = b.term_min;
  for (int i = 0; i < 2; i++) {
    out->witness_max[i] = b.witness_max[i];
    out->witness_min[i] = b.witness_min[i];
  }
  out->kblock = b.kblock;
}

int mmp_int8_bound(uint64_t p, int entry_bits, mmp_int8_bound_t* out) {
  if (!out) return MMP_EINVAL;
  if (p != 0 && entry_bits == 0 && p >= 5 && p < mmp::kPMax) {
    copy_bound(mmp::int8_bound_residues(p), out);
    return MMP_OK;
  }
  if (p == 0 && entry_bits >= 1 && entry_bits <= 62) {
    copy_bound(mmp::int8_bound_integers(entry_bits), out);
    return MMP_OK;
  }
  return MMP_EINVAL;
}

int mmp_int8_interval_bound(int digits, int64_t lo, int64_t hi, mmp_int8_bound_t* out) {
  if (!out || digits < 1 || digits > 8 || lo > hi) return MMP_EINVAL;
  const __int128 top = mmp::radix_top(digits), R = top / 127;  // 127 R, R = (256^D - 1) / 255
  if ((__int128)hi > top || (__int128)lo < -128 * R) return MMP_EINVAL;
  copy_bound(mmp::int8_bound_interval(digits, lo, hi), out);
  return MMP_OK;
}

size_t mmp_footprint(const mmp_job* job, const mmp_plan_t* plan) {
  if (!job || job->m < 0 || job->n < 0 || job->k < 0) return 0;
  const size_t m = (size_t)job->m, n = (size_t)job->n, k = (size_t)job->k;
  size_t bytes = 8 * (m * k + k * n + m * n);
  if (plan) {
    if (plan->form == MMP_FORM_INT8_WORDS)
      bytes += mmp::int8_planes_bytes(plan->digits_a, job->m, job->n, job->k, false, false);
    else
      bytes += 8 * ((size_t)plan->u * m * k + (size_t)plan->v * k * n);
  }
  return bytes;
}

int mm_modp_async(const mmp_opts* opts, uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                  void* stream) {
  try {
    if (int st = check_product_args(m, n, k, A, lda, B, ldb, C, ldc)) return st;
    if (opts && opts->batch_launch) return MMP_EINVAL;  // a batch option
    const mmp_operand_t* pa = opts ? opts->prepared_a : nullptr;
    const mmp_operand_t* pb = opts ? opts->prepared_b : nullptr;
    mmp_plan_t pl;
    if (pa || pb) {
      // prepared digit planes: the INT8 form, planned without them
      if (u != 0 || opts->form == MMP_FORM_FP64_WORDS || opts->tile || opts->extended_block ||
          opts->centered_words)
        return MMP_EINVAL;
      mmp_opts o2 = *opts;
      o2.form = MMP_FORM_INT8_WORDS;
      o2.prepared_a = nullptr;
      o2.prepared_b = nullptr;
      if (int st = mmp::plan(p, 0, 0, m, n, k, &o2, &pl)) return st;
      if (pa && !operand_fits(*pa, 0, p, m, k, pl.digits_a)) return MMP_EINVAL;
      if (pb && !operand_fits(*pb, 1, p, k, n, pl.digits_b)) return MMP_EINVAL;
    } else if (int st = mmp::plan(p, u, v, m, n, k, opts, &pl)) {
      return st;
    }
    if (!fp64_ld_ok(pl, lda, ldb)) {
      // leading dimensions beyond the FP64 kernel's offsets: an AUTO plan
      // takes the INT8 form, which has no such limit; a forced one fails
      if (u != 0 || (opts && (opts->form != MMP_FORM_AUTO || opts->tile || opts->force_kblock ||
                              opts->extended_block || opts->centered_words)))
        return MMP_EINVAL;
      mmp_opts o2;
      std::memset(&o2, 0, sizeof(o2));
      if (opts) o2 = *opts;
      o2.form = MMP_FORM_INT8_WORDS;
      if (int st = mmp::plan(p, 0, 0, m, n, k, &o2, &pl)) return st;
    }
    if (m == 0 || n == 0) return MMP_OK;
    if (k == 0) return hip_status(launch_zero_fill(C, m, n, ldc, stream));
    if (opts && opts->validate_entries)
      if (int st = validate_product_entries(p, m, n, k, A, lda, B, ldb, stream)) return st;

    // split-K residues go after the digit planes made per call (INT8) or
    // fill the workspace (FP64)
    const size_t planes = pl.form == MMP_FORM_INT8_WORDS
                              ? int8_planes_bytes(pl.digits_a, m, n, k, pa != nullptr, pb != nullptr) : 0;
    const size_t need = planes + (pl.splits > 1 ? 8 * (size_t)pl.splits * (size_t)m * (size_t)n : 0);
    void* work = nullptr;
    bool owned = false;
    if (int st = acquire_workspace(need, opts, stream, &work, &owned)) return st;
    double* partial = pl.splits > 1 ? (double*)((char*)work + planes) : nullptr;
    int e;
    if (pl.form == MMP_FORM_INT8_WORDS) {
      Int8Args g = make_int8_args(pl, m, n, k, A, lda, B, ldb, C, ldc, (int8_t*)work);
      g.resident_a = pa ? pa->planes : nullptr;
      g.resident_b = pb ? pb->planes : nullptr;
      g.splits = pl.splits;
      g.partial = partial;
      e = launch_int8_digitize(pl.digits_a, g, stream);
      if (!e) e = launch_int8_gemm(pl.digits_a, &g, 1, stream);
    } else {
      Fp64Batch b;
      std::memset(&b, 0, sizeof(b));
      b.njobs = 1;
      b.job[0] = make_fp64_args(pl, m, n, k, A, lda, B, ldb, C, ldc);
      b.job[0].splits = pl.splits;
      b.job[0].partial = partial;
      e = launch_fp64_words(pl.u, pl.v, pl.tile, b, stream);
    }
    if (!e && pl.splits > 1) e = launch_splitk_reduce(partial, pl.splits, m, n, (double)p, C, ldc, stream);
    const int st = hip_status(e);
    const int st2 = release_workspace(work, owned, stream);
    return st ? st : st2;
  } catch (...) {
    return MMP_EINVAL;
  }
}

size_t mmp_operand_bytes(uint64_t p, int side, int64_t rows, int64_t cols) {
  if (p < 5 || p >= kPMax || (side != 0 && side != 1) || rows <= 0 || cols <= 0) return 0;
  const int64_t inner = side == 0 ? cols : rows, outer = side == 0 ? rows : cols;
  return digit_planes_bytes(digits_for(p), outer, (inner + 63) / 64 * 64);
}

int mmp_prepare_operand(uint64_t p, int side, const double* M, int64_t rows, int64_t cols, int64_t ld,
                        void* planes, size_t planes_bytes, mmp_operand_t* out, void* stream) {
  try {
    const size_t need = mmp_operand_bytes(p, side, rows, cols);
    if (!out || !M || !planes || need == 0 || ld < cols || planes_bytes < need) return MMP_EINVAL;
    if (ranges_overlap(planes, need, M, span_bytes(rows, cols, ld))) return MMP_EINVAL;
    const int64_t inner = side == 0 ? cols : rows;
    mmp_operand_t o;
    std::memset(&o, 0, sizeof(o));
    o.planes = (const int8_t*)planes;
    o.p = p;
    o.side = side;
    o.digits = digits_for(p);
    o.rows = rows;
    o.cols = cols;
    o.kp = (inner + 63) / 64 * 64;
    if (int e = launch_int8_digitize_side(o.digits, side, M, rows, cols, ld, o.kp, p, (int8_t*)planes, stream))
      return hip_status(e);
    *out = o;
    return MMP_OK;
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
