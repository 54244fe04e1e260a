// Host-only exercise of the library for sanitizer builds (AddressSanitizer +
// UndefinedBehaviorSanitizer, ThreadSanitizer).  Test infrastructure: it
// touches no GPU.  It drives the planner, the INT8 block bound, the
// footprint, the argument checks of the product entry points (refused on the
// host before any device call) and a dry-run request server fed by several
// submitting threads, with one more server whose launches fail on the host.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "mmp.h"

static int failures = 0;
#define EXPECT(c)                                                      \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #c); \
      failures++;                                                      \
    }                                                                  \
  } while (0)

static void planner() {
  const uint64_t primes[] = {5, 7, 251, 65521, 1048573, 8388593, 33554393, 67108859, 2147483647ull,
                             68719476731ull, 1099511627689ull, 1125899906842597ull, 4503599627370449ull};
  const int64_t shapes[][3] = {{0, 0, 0}, {1, 1, 1}, {17, 5, 3}, {512, 512, 512}, {4096, 4096, 4096},
                               {16384, 16384, 256}, {512, 512, 131072}, {10923, 32, 32768}};
  for (uint64_t p : primes)
    for (auto& s : shapes)
      for (int u = 0; u <= 4; u++)
        for (int v = 0; v <= 4; v++) {
          if ((u == 0) != (v == 0)) continue;
          for (int form = 0; form <= 2; form++)
            for (int variant = 0; variant < 4; variant++) {
              mmp_opts o;
              std::memset(&o, 0, sizeof(o));
              o.form = form;
              o.extended_block = variant == 1;
              o.centered_words = variant == 2;
              o.strict_fmod = variant == 3;
              mmp_plan_t pl;
              const int st = mmp_plan(p, u, v, s[0], s[1], s[2], &o, &pl);
              EXPECT(st <= 0);
              if (st == MMP_OK) {
                mmp_job j;
                std::memset(&j, 0, sizeof(j));
                j.p = p;
                j.m = s[0];
                j.n = s[1];
                j.k = s[2];
                EXPECT(mmp_footprint(&j, &pl) >= (size_t)(8 * (s[0] * s[1])));
              }
            }
        }
  for (int st = 0; st >= -9; st--) EXPECT(mmp_strerror(st) != nullptr);
}

static void int8_bounds() {
  for (uint64_t p = 5; p < 70000; p += 997) {
    mmp_int8_bound_t b;
    EXPECT(mmp_int8_bound(p, 0, &b) == MMP_OK);
    EXPECT(b.kblock % 64 == 0 && b.kblock > 0);
  }
  for (int bits = 1; bits <= 62; bits++) {
    mmp_int8_bound_t b;
    EXPECT(mmp_int8_bound(0, bits, &b) == MMP_OK);
  }
  mmp_int8_bound_t b;
  EXPECT(mmp_int8_bound(0, 63, &b) == MMP_EINVAL);
  EXPECT(mmp_int8_interval_bound(9, 0, 1, &b) == MMP_EINVAL);
  EXPECT(mmp_int8_interval_bound(8, INT64_MIN, INT64_MAX, &b) == MMP_EINVAL);
  EXPECT(mmp_int8_interval_bound(3, -100, 100, &b) == MMP_OK);
}

static void argument_errors() {
  double* fake = (double*)(uintptr_t)0x10000;
  double* fake2 = (double*)(uintptr_t)0x20000000;
  double* fake3 = (double*)(uintptr_t)0x40000000;
  EXPECT(mm_modp_async(nullptr, 3, 0, 0, 4, 4, 4, fake, 4, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  EXPECT(mm_modp_async(nullptr, 1ull << 52, 0, 0, 4, 4, 4, fake, 4, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  EXPECT(mm_modp_async(nullptr, 65521, 0, 0, -1, 4, 4, fake, 4, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  EXPECT(mm_modp_async(nullptr, 65521, 0, 0, 4, 4, 4, fake, 3, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  EXPECT(mm_modp_async(nullptr, 65521, 5, 1, 4, 4, 4, fake, 4, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  mmp_opts o;
  std::memset(&o, 0, sizeof(o));
  o.validate_entries = 1;
  EXPECT(mm_modp_static(&o, 65521, 0, 0, 4, 4, 4, fake, 4, fake2, 4, fake3, 4, nullptr) == MMP_EINVAL);
  std::memset(&o, 0, sizeof(o));
  o.form = MMP_FORM_INT8_WORDS;
  o.splits = 1;
  EXPECT(mm_modp_static(&o, 4503599627370449ull, 0, 0, 16384, 16384, 4096, fake, 4096, fake2, 16384, fake3,
                        16384, nullptr) == MMP_ENOMEM);
  mmp_job jobs[2];
  std::memset(jobs, 0, sizeof(jobs));
  EXPECT(mm_modp_batched(jobs, -1, nullptr, nullptr) == MMP_EINVAL);
  uint64_t primes[1] = {4};
  double* outs[1] = {fake3};
  EXPECT(mm_modp_crt(nullptr, (const uint64_t*)fake, 4, (const uint64_t*)fake2, 4, 4, 4, 4, 20, primes, 1, outs, 4,
                     nullptr) == MMP_EINVAL);
}

static void dry_run_server() {
  mmp_server* srv = nullptr;
  EXPECT(mmp_server_create(&srv, 0, (size_t)8 << 30, 16, MMP_SERVER_DRY_RUN) == MMP_OK);
  if (!srv) return;
  const int nthreads = 4, per = 150;
  std::vector<std::vector<uint64_t>> tickets(nthreads);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; t++) {
    th.emplace_back([&, t] {
      for (int i = 0; i < per; i++) {
        mmp_job j;
        std::memset(&j, 0, sizeof(j));
        j.p = (i % 3 == 0) ? 1125899906842597ull : (i % 3 == 1) ? 2147483647ull : 65521;
        j.m = 32 + (i * 7 + t) % 200;
        j.n = 16 + (i * 13) % 150;
        j.k = 8 + (i * 29 + 3 * t) % 700;
        const uintptr_t base = (uintptr_t)0x10000000 * (uintptr_t)(1 + t) + (uintptr_t)i * 0x100000;
        j.A = (const double*)base;
        j.lda = j.k;
        j.B = (const double*)(base + 8 * j.m * j.k + 4096);
        j.ldb = j.n;
        j.C = (double*)(base + 8 * (j.m * j.k + j.k * j.n) + 8192);
        j.ldc = j.n;
        uint64_t tk = 0;
        const int st = (i % 2) ? mmp_submit(srv, &j, 0, &tk) : mmp_submit_after(srv, &j, 0, nullptr, &tk);
        EXPECT(st == MMP_OK);
        if (st == MMP_OK) tickets[t].push_back(tk);
        if (i % 10 == 0) {
          mmp_server_stats_t s;
          EXPECT(mmp_server_stats(srv, &s) == MMP_OK);
        }
      }
      for (uint64_t tk : tickets[t]) {
        int status = -100;
        double lat = -1;
        EXPECT(mmp_wait(srv, tk, 60.0, &status, &lat) == MMP_OK);
        EXPECT(status == MMP_OK && lat >= 0);
      }
    });
  }
  for (auto& x : th) x.join();
  mmp_server_stats_t s;
  EXPECT(mmp_server_stats(srv, &s) == MMP_OK);
  EXPECT(s.completed == nthreads * per && s.failed == 0 && s.used_bytes == 0);
  EXPECT(mmp_server_destroy(srv) == MMP_OK);

  // launches that fail on the host: waiters wake with the error
  EXPECT(mmp_server_create(&srv, 0, (size_t)1 << 30, 4, MMP_SERVER_DRY_RUN | MMP_SERVER_FAIL_LAUNCHES) == MMP_OK);
  if (!srv) return;
  std::vector<std::thread> w;
  for (int t = 0; t < 3; t++) {
    w.emplace_back([&, t] {
      mmp_job j;
      std::memset(&j, 0, sizeof(j));
      j.p = 65521;
      j.m = j.n = j.k = 64;
      const uintptr_t base = (uintptr_t)0x10000000 * (uintptr_t)(1 + t);
      j.A = (const double*)base;
      j.lda = 64;
      j.B = (const double*)(base + 65536);
      j.ldb = 64;
      j.C = (double*)(base + 2 * 65536);
      j.ldc = 64;
      uint64_t tk = 0;
      EXPECT(mmp_submit(srv, &j, 0, &tk) == MMP_OK);
      int status = 0;
      double lat = 0;
      EXPECT(mmp_wait(srv, tk, -1.0, &status, &lat) == MMP_OK);
      EXPECT(status == MMP_ENOMEM);
    });
  }
  for (auto& x : w) x.join();
  EXPECT(mmp_server_destroy(srv) == MMP_OK);
}

int main() {
  planner();
  int8_bounds();
  argument_errors();
  dry_run_server();
  std::printf("host driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
