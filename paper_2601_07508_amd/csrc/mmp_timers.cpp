// Phase timers: optional start/stop events attached to every kernel launch
// (hipExtLaunchKernelGGL records them with the dispatch itself, so they time
// the kernel and not the queue around it), summed per phase name.  Off by
// default; when off the hooks cost one atomic load.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mmp_internal.h"

namespace {

struct Pending {
  std::string name;
  hipEvent_t e0, e1;
};
struct Sum {
  int64_t launches = 0;
  double ms = 0.0;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::map<std::string, Sum> g_sums;

void drain_locked() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      Sum& s = g_sums[p.name];
      s.launches += 1;
      s.ms += ms;
    }
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  g_pending.clear();
}

}  // namespace

namespace mmp {

TimerTok* timer_begin(const char* phase) {
  if (!g_on.load(std::memory_order_relaxed)) return nullptr;
  auto* t = new TimerTok{nullptr, nullptr, phase};
  if (hipEventCreate(&t->e0) != hipSuccess || hipEventCreate(&t->e1) != hipSuccess) {
    if (t->e0) (void)hipEventDestroy(t->e0);
    if (t->e1) (void)hipEventDestroy(t->e1);
    delete t;
    return nullptr;
  }
  return t;
}

void timer_commit(TimerTok* t, int launch_status) {
  if (!t) return;
  if (launch_status == 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back(Pending{t->name, t->e0, t->e1});
  } else {
    (void)hipEventDestroy(t->e0);
    (void)hipEventDestroy(t->e1);
  }
  delete t;
}

}  // namespace mmp

extern "C" {

int mmp_timers_enable(int on) {
  g_on.store(on ? 1 : 0);
  return MMP_OK;
}

int mmp_timers_read(mmp_timer* out, int cap, int reset) {
  if (cap < 0 || (cap > 0 && !out)) return MMP_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  int n = 0;
  for (auto& kv : g_sums) {
    if (n < cap) {
      std::memset(&out[n], 0, sizeof(mmp_timer));
      std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.launches;
      out[n].total_ms = kv.second.ms;
    }
    n++;
  }
  if (reset) g_sums.clear();
  return n;
}

}  // extern "C"
