// Batched products and multi-modular (CRT) products.
//
// mm_modp_batched: every product is planned on its own; products that share
// a kernel configuration run together, up to kMaxBatch per launch, with the
// job table in the kernel arguments.  INT8-form products first get their
// digit planes (one workspace for the whole batch), then one digit GEMM per
// digit count.  The batch is enqueued on one stream with no host
// synchronisation, so with a caller workspace it can be captured into a HIP
// graph and replayed.
//
// mm_modp_crt: one integer pair A, B against many moduli.  When k fits one
// exact int32 block the integers are digitised once, one digit GEMM forms
// the digit-weight sums of A B, and each modulus reduces those sums in the
// epilogue; otherwise A and B are reduced mod each p on the device and the
// products run as a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "mmp_internal.h"

namespace {

using namespace mmp;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Planned {
  const mmp_job* job;
  mmp_plan_t plan;
  size_t ws_offset;
};

int plan_batch(const mmp_job* jobs, int count, const mmp_opts* opts, std::vector<Planned>* out,
               size_t* ws_total) {
  if (count < 0 || (count > 0 && !jobs)) return MMP_EINVAL;
  // batched products run one k-range each (their many tiles fill the chip)
  mmp_opts o1;
  std::memset(&o1, 0, sizeof(o1));
  if (opts) o1 = *opts;
  o1.splits = 1;
  opts = &o1;
  out->clear();
  out->reserve(count);
  size_t ws = 0;
  for (int i = 0; i < count; i++) {
    const mmp_job& j = jobs[i];
    if (int st = check_product_args(j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc)) return st;
    Planned pj;
    pj.job = &j;
    if (int st = mmp::plan(j.p, j.u, j.v, j.m, j.n, j.k, opts, &pj.plan)) return st;
    if (!fp64_ld_ok(pj.plan, j.lda, j.ldb)) return MMP_EINVAL;
    pj.ws_offset = ws;
    if (pj.plan.form == MMP_FORM_INT8_WORDS && j.m > 0 && j.n > 0 && j.k > 0)
      ws += align_up(pj.plan.workspace_bytes);
    out->push_back(pj);
  }
  // outputs must not overlap each other
  for (int a = 0; a < count; a++)
    for (int b = a + 1; b < count; b++)
      if (ranges_overlap(jobs[a].C, span_bytes(jobs[a].m, jobs[a].n, jobs[a].ldc), jobs[b].C,
                         span_bytes(jobs[b].m, jobs[b].n, jobs[b].ldc)))
        return MMP_EINVAL;
  *ws_total = ws;
  return MMP_OK;
}

int run_batch(const std::vector<Planned>& pj, const mmp_opts* opts, size_t ws_total, void* stream) {
  const bool validate = opts && opts->validate_entries;
  // zero fills, validation
  for (const Planned& x : pj) {
    const mmp_job& j = *x.job;
    if (j.m == 0 || j.n == 0) continue;
    if (j.k == 0) {
      if (int e = launch_zero_fill(j.C, j.m, j.n, j.ldc, stream)) return hip_status(e);
      continue;
    }
    if (validate)
      if (int st = validate_product_entries(j.p, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, stream)) return st;
  }
  // FP64-word products, grouped by kernel configuration
  std::map<std::tuple<int, int, int, int>, std::vector<const Planned*>> groups;
  for (const Planned& x : pj) {
    const mmp_job& j = *x.job;
    if (j.m == 0 || j.n == 0 || j.k == 0 || x.plan.form != MMP_FORM_FP64_WORDS) continue;
    groups[std::make_tuple(x.plan.u, x.plan.v, x.plan.tile, fp64_class(x.plan.slots, x.plan.kblock, x.plan.lazy != 0))].push_back(&x);
  }
  for (auto& kv : groups) {
    const auto& v = kv.second;
    for (size_t c = 0; c < v.size(); c += kMaxBatch) {
      Fp64Batch b;
      std::memset(&b, 0, sizeof(b));
      b.njobs = (int)std::min<size_t>(kMaxBatch, v.size() - c);
      for (int t = 0; t < b.njobs; t++) {
        const Planned& x = *v[c + t];
        const mmp_job& j = *x.job;
        b.job[t] = make_fp64_args(x.plan, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc);
      }
      if (int e = launch_fp64_words(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), b,
                                    stream))
        return hip_status(e);
    }
  }
  // INT8-digit products
  if (ws_total == 0) return MMP_OK;
  void* work = nullptr;
  bool owned = false;
  if (int st = acquire_workspace(ws_total, opts, stream, &work, &owned)) return st;
  int err = 0;
  // the one-launch form: planes of up to 64 products in one launch, their
  // digit GEMM in one persistent launch
  const int mode = opts ? opts->batch_launch : 0;
  std::vector<Int8Args> all;
  std::vector<int> all_digits;
  for (const Planned& x : pj) {
    const mmp_job& j = *x.job;
    if (j.m == 0 || j.n == 0 || j.k == 0 || x.plan.form != MMP_FORM_INT8_WORDS) continue;
    all.push_back(make_int8_args(x.plan, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc,
                                 (int8_t*)work + x.ws_offset));
    all_digits.push_back(x.plan.digits_a);
  }
  if (mode == 2 || (mode == 0 && all.size() >= 2)) {
    for (size_t c = 0; c < all.size() && !err; c += kMaxMixedBatch) {
      const int nj = (int)std::min<size_t>(kMaxMixedBatch, all.size() - c);
      err = launch_int8_batch(all.data() + c, all_digits.data() + c, nj, stream);
    }
    const int st = hip_status(err);
    const int st2 = release_workspace(work, owned, stream);
    return st ? st : st2;
  }
  std::map<int, std::vector<Int8Args>> by_digits;
  for (const Planned& x : pj) {
    const mmp_job& j = *x.job;
    if (j.m == 0 || j.n == 0 || j.k == 0 || x.plan.form != MMP_FORM_INT8_WORDS) continue;
    Int8Args g = make_int8_args(x.plan, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc,
                                (int8_t*)work + x.ws_offset);
    if (!err) err = launch_int8_digitize(x.plan.digits_a, g, stream);
    by_digits[x.plan.digits_a].push_back(g);
  }
  for (auto& kv : by_digits) {
    for (size_t c = 0; c < kv.second.size() && !err; c += kMaxBatch) {
      const int nj = (int)std::min<size_t>(kMaxBatch, kv.second.size() - c);
      err = launch_int8_gemm(kv.first, kv.second.data() + c, nj, stream);
    }
  }
  const int st = hip_status(err);
  const int st2 = release_workspace(work, owned, stream);
  return st ? st : st2;
}

// CRT: workspace for the fast path, or for the reduced copies of the
// fallback (two binary64 matrices per modulus plus their products' needs).
bool crt_fast(int64_t k, int entry_bits, int nprimes) {
  return k <= int8_bound_integers(entry_bits).kblock && nprimes >= 1;
}

}  // namespace

extern "C" {

size_t mmp_workspace_batched(const mmp_job* jobs, int count, const mmp_opts* opts) {
  std::vector<Planned> pj;
  size_t ws = 0;
  if (plan_batch(jobs, count, opts, &pj, &ws) != MMP_OK) return 0;
  return ws;
}

int mm_modp_batched(const mmp_job* jobs, int count, const mmp_opts* opts, void* stream) {
  try {
    std::vector<Planned> pj;
    size_t ws = 0;
    if (int st = plan_batch(jobs, count, opts, &pj, &ws)) return st;
    return run_batch(pj, opts, ws, stream);
  } catch (...) {
    return MMP_EINVAL;
  }
}

size_t mmp_workspace_crt(int64_t m, int64_t n, int64_t k, int entry_bits, int nprimes, const mmp_opts* opts) {
  (void)opts;
  if (m <= 0 || n <= 0 || k <= 0 || entry_bits < 1 || entry_bits > 62 || nprimes < 1) return 0;
  const int d = crt_digits(entry_bits);
  const size_t kp = (size_t)((k + 63) / 64 * 64);
  if (crt_fast(k, entry_bits, nprimes)) return digit_planes_bytes(d, m, kp) + digit_planes_bytes(d, n, kp);
  // fallback: per modulus, reduced A and B in binary64 (the products use the
  // planner's form; an INT8 product needs at most 7-digit planes of A and B)
  const size_t per = align_up(8 * (size_t)(m * k + k * n)) + align_up(int8_workspace_bytes(kMaxDigits, m, n, k));
  return per * (size_t)nprimes;
}

int mm_modp_crt(const mmp_opts* opts, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb, int64_t m,
                int64_t n, int64_t k, int entry_bits, const uint64_t* primes, int nprimes, double* const* C,
                int64_t ldc, void* stream) {
  try {
    if (m < 0 || n < 0 || k < 0 || entry_bits < 1 || entry_bits > 62) return MMP_EINVAL;
    if (nprimes < 1 || !primes || !C) return MMP_EINVAL;
    if (opts) {
      if (opts->batch_launch != 0) return MMP_EINVAL;
      if (opts->prepared_a || opts->prepared_b) return MMP_EINVAL;
    }
    for (int i = 0; i < nprimes; i++) {
      if (primes[i] < 5 || primes[i] >= kPMax) return MMP_EINVAL;
      if (m > 0 && n > 0 && !C[i]) return MMP_EINVAL;
    }
    if (m == 0 || n == 0) return MMP_OK;
    if (ldc < n) return MMP_EINVAL;
    if (k > 0 && (!A || !B || lda < k || ldb < n)) return MMP_EINVAL;
    for (int i = 0; i < nprimes; i++)
      for (int j = i + 1; j < nprimes; j++)
        if (ranges_overlap(C[i], span_bytes(m, n, ldc), C[j], span_bytes(m, n, ldc))) return MMP_EINVAL;
    if (k == 0) {
      for (int i = 0; i < nprimes; i++)
        if (int e = launch_zero_fill(C[i], m, n, ldc, stream)) return hip_status(e);
      return MMP_OK;
    }
    if (opts && opts->validate_entries)
      if (int st = validate_integer_entries(entry_bits, m, n, k, A, lda, B, ldb, stream)) return st;

    const int d = crt_digits(entry_bits);
    const size_t ws = mmp_workspace_crt(m, n, k, entry_bits, nprimes, opts);
    void* work = nullptr;
    bool owned = false;
    if (int st = acquire_workspace(ws, opts, stream, &work, &owned)) return st;
    int st = MMP_OK;
    if (crt_fast(k, entry_bits, nprimes)) {
      CrtLaunch c;
      std::memset(&c, 0, sizeof(c));
      c.A = A;
      c.B = B;
      c.m = m;
      c.n = n;
      c.k = k;
      c.lda = lda;
      c.ldb = ldb;
      c.ldc = ldc;
      c.kp = (k + 63) / 64 * 64;
      c.work = (int8_t*)work;
      for (int i0 = 0; i0 < nprimes && st == MMP_OK; i0 += kMaxPrimesCrt) {
        c.nprimes = std::min(kMaxPrimesCrt, nprimes - i0);
        for (int i = 0; i < c.nprimes; i++) {
          c.p[i] = primes[i0 + i];
          c.C[i] = C[i0 + i];
        }
        st = hip_status(launch_crt(d, c, stream));
      }
    } else {
      // reduce mod each p on the device, then the products as one batch
      const size_t per = align_up(8 * (size_t)(m * k + k * n)) + align_up(int8_workspace_bytes(kMaxDigits, m, n, k));
      std::vector<mmp_job> jobs(nprimes);
      for (int i = 0; i < nprimes && st == MMP_OK; i++) {
        double* Ar = (double*)((char*)work + per * i);
        double* Br = Ar + m * k;
        st = hip_status(launch_reduce_mod(A, m, k, lda, primes[i], Ar, k, stream));
        if (st == MMP_OK) st = hip_status(launch_reduce_mod(B, k, n, ldb, primes[i], Br, n, stream));
        mmp_job& j = jobs[i];
        std::memset(&j, 0, sizeof(j));
        j.p = primes[i];
        j.m = m;
        j.n = n;
        j.k = k;
        j.A = Ar;
        j.lda = k;
        j.B = Br;
        j.ldb = n;
        j.C = C[i];
        j.ldc = ldc;
      }
      // each product's digit planes go after its reduced copies
      for (int i = 0; i < nprimes && st == MMP_OK; i++) {
        mmp_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o.form = opts->form;
        o.splits = 1;
        o.workspace = (char*)work + per * i + align_up(8 * (size_t)(m * k + k * n));
        o.workspace_bytes = align_up(int8_workspace_bytes(kMaxDigits, m, n, k));
        st = mm_modp_async(&o, jobs[i].p, 0, 0, m, n, k, jobs[i].A, jobs[i].lda, jobs[i].B, jobs[i].ldb,
                           jobs[i].C, jobs[i].ldc, stream);
      }
    }
    const int st2 = release_workspace(work, owned, stream);
    return st ? st : st2;
  } catch (...) {
    return MMP_EINVAL;
  }
}

}  // extern "C"
