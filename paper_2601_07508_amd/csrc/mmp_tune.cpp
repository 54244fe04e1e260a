// Autotuner: times the candidate plans of one product shape on the device
// and caches the fastest for its class (bitsize of p; ceil(log2) of m, n, k).
// Candidates: every word pair the paper's bound admits (Section 3.3) with
// each tile shape and the planner's block for it (paper or, when allowed,
// extended bound; with centered words, every pair the centered bound
// admits), and the INT8-digit form unless a word-form option is set.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "mmp_internal.h"

namespace {
using namespace mmp;

struct Cand {
  int form, u, v, tile;
  int64_t kblock;
};

}  // namespace

extern "C" {

int mmp_autotune(uint64_t p, int64_t m, int64_t n, int64_t k, const mmp_opts* opts, mmp_plan_t* best,
                 int* tried) {
  try {
    if (!best || m <= 0 || n <= 0 || k <= 0) return MMP_EINVAL;
    if (tried) *tried = 0;
    mmp_opts base;
    std::memset(&base, 0, sizeof(base));
    if (opts) base = *opts;
    const bool extended = base.extended_block != 0;
    const bool centered = base.centered_words != 0;
    if (base.form != MMP_FORM_AUTO || base.force_kblock || base.tile) return MMP_EINVAL;
    mmp_plan_t probe;
    if (int st = plan(p, 0, 0, m, n, k, &base, &probe)) return st;  // validates p and sizes

    // candidate list
    std::vector<Cand> cands;
    static const int pairs[][2] = {{1, 1}, {1, 2}, {2, 1}, {1, 3}, {3, 1}, {2, 2},
                                   {1, 4}, {4, 1}, {2, 3}, {3, 2}, {2, 4}, {4, 2}};
    for (auto& pr : pairs) {
      if ((centered ? centered_lambda(p, pr[0], pr[1]) : paper_lambda(p, pr[0], pr[1])) < 1) continue;
      for (int tile = 1; tile <= 3; tile++) {
        mmp_opts o = base;
        o.form = MMP_FORM_FP64_WORDS;
        o.tile = tile;
        mmp_plan_t pl;
        if (plan(p, pr[0], pr[1], m, n, k, &o, &pl) == MMP_OK)
          cands.push_back({MMP_FORM_FP64_WORDS, pr[0], pr[1], tile, pl.kblock});
      }
    }
    if (!extended && !centered) cands.push_back({MMP_FORM_INT8_WORDS, 0, 0, 0, 0});

    // scratch operands and output
    double *A = nullptr, *B = nullptr, *C = nullptr;
    const size_t bytes = 8 * (size_t)(m * k + k * n + m * n);
    if (int e = (int)hipMalloc(&A, bytes)) return hip_status(e);
    B = A + m * k;
    C = B + k * n;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int err = (int)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (!err) err = (int)hipEventCreate(&e0);
    if (!err) err = (int)hipEventCreate(&e1);
    if (!err) err = launch_fill_mod(A, m * k, p, 1, s);
    if (!err) err = launch_fill_mod(B, k * n, p, 2, s);
    Cand win{0, 0, 0, 0, 0};
    double win_ms = 1e300;
    for (size_t i = 0; i < cands.size() && !err; i++) {
      const Cand& c = cands[i];
      mmp_opts o = base;
      o.form = c.form;
      o.tile = c.tile;
      o.force_kblock = c.form == MMP_FORM_FP64_WORDS ? c.kblock : 0;
      auto once = [&]() {
        return mm_modp_async(&o, p, c.u, c.v, m, n, k, A, k, B, n, C, n, s);
      };
      int st = once();  // warm-up (also loads the kernel)
      if (st != MMP_OK) continue;
      // repeat so that a measurement spans at least a few milliseconds
      int reps = 1;
      float ms = 0;
      for (int round = 0; round < 2 && !err; round++) {
        err = (int)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == MMP_OK; r++) st = once();
        if (!err) err = (int)hipEventRecord(e1, s);
        if (!err) err = (int)hipEventSynchronize(e1);
        if (!err) err = (int)hipEventElapsedTime(&ms, e0, e1);
        if (st != MMP_OK) break;
        if (round == 0) reps = ms > 0 ? (int)std::min(50.0, std::max(1.0, 5.0 / ms)) : 50;
      }
      if (st != MMP_OK || err) continue;
      const double per = ms / reps;
      if (tried) (*tried)++;
      if (per < win_ms) {
        win_ms = per;
        win = c;
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(A);
    if (err) return hip_status(err);
    if (win_ms >= 1e299) return MMP_EBOUND;
    tune_store(p, m, n, k, centered ? 2 : extended ? 1 : 0, TunedChoice{win.form, win.u, win.v, win.tile, win.kblock, win_ms});
    return plan(p, 0, 0, m, n, k, &base, best);
  } catch (...) {
    return MMP_ENOMEM;
  }
}

int mmp_tune_cache_clear(void) {
  tune_clear();
  return MMP_OK;
}

int mmp_tune_cache_save(const char* path) { return path ? tune_save(path) : MMP_EINVAL; }

int mmp_tune_cache_load(const char* path) { return path ? tune_load(path) : MMP_EINVAL; }

}  // extern "C"
