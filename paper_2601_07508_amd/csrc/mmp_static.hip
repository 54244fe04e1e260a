// mm_modp_static: the asynchronous product with no allocation at all.  Its
// workspace (the INT8 form's digit planes, split-K residues) is a file-scope
// device array of fixed size, one per device, instead of stream-ordered pool
// memory, for callers that cannot allocate (code under HIP graph capture,
// serving loops that must not touch the allocator).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <vector>

#include "mmp_internal.h"

namespace {

// Each device that loads the library holds its own copy until the process
// ends.  In host code this name is only a handle for hipGetSymbolAddress:
// kernels receive the device address it returns.
__device__ __align__(256) unsigned char scratch[MMP_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
std::vector<void*> g_addr;  // per device: the address of that device's array

// The array's address on the current device, looked up once per device.
int scratch_address(void** out) {
  int dev = 0;
  if (int e = (int)hipGetDevice(&dev)) return mmp::hip_status(e);
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_addr.size() <= dev) g_addr.resize(dev + 1, nullptr);
  if (!g_addr[dev]) {
    void* p = nullptr;
    if (int e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return mmp::hip_status(e);
    if (!p) return MMP_EHIP;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return MMP_OK;
}

}  // namespace

extern "C" int mm_modp_static(const mmp_opts* opts, uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k,
                              const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                              void* stream) {
  try {
    mmp_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    // the caller's workspace would replace the array, and validation needs a
    // device flag of its own: neither belongs to this entry point
    if (o.workspace || o.workspace_bytes || o.validate_entries) return MMP_EINVAL;
    if (int st = mmp::check_product_args(m, n, k, A, lda, B, ldb, C, ldc)) return st;
    // the plan mm_modp_async makes (the same planner call on the same options)
    mmp_plan_t pl;
    if (o.prepared_a || o.prepared_b) {
      mmp_opts o2 = o;
      o2.form = MMP_FORM_INT8_WORDS;
      o2.prepared_a = nullptr;
      o2.prepared_b = nullptr;
      if (int st = mmp::plan(p, 0, 0, m, n, k, &o2, &pl)) return st;
    } else if (int st = mmp::plan(p, u, v, m, n, k, &o, &pl)) {
      return st;
    }
    if (!mmp::fp64_ld_ok(pl, lda, ldb)) {  // mm_modp_async's fallback to the INT8 form
      mmp_opts o2 = o;
      o2.form = MMP_FORM_INT8_WORDS;
      if (mmp::plan(p, 0, 0, m, n, k, &o2, &pl) != MMP_OK) return MMP_EINVAL;
    }
    const size_t planes = pl.form == MMP_FORM_INT8_WORDS
                              ? mmp::int8_planes_bytes(pl.digits_a, m, n, k, o.prepared_a != nullptr,
                                                       o.prepared_b != nullptr)
                              : 0;
    const size_t need = planes + (pl.splits > 1 ? 8 * (size_t)pl.splits * (size_t)m * (size_t)n : 0);
    if (need > (size_t)MMP_STATIC_SCRATCH_BYTES) return MMP_ENOMEM;
    void* ptr = nullptr;
    if (need > 0)
      if (int st = scratch_address(&ptr)) return st;
    o.workspace = ptr;
    o.workspace_bytes = ptr ? (size_t)MMP_STATIC_SCRATCH_BYTES : 0;
    return mm_modp_async(&o, p, u, v, m, n, k, A, lda, B, ldb, C, ldc, stream);
  } catch (...) {
    return MMP_EINVAL;
  }
}
