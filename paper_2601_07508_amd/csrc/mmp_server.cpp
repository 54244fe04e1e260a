// Request server: modular products of mixed shapes and moduli, served as
// they arrive, with continuous batching.
//
// A scheduler thread owns the device work:
//   - admission: requests are admitted in arrival order while a request slot
//     is free and the device footprint of everything in flight (operands,
//     result and word or digit copies, Section 3.3's storage cost; resident
//     operands counted once at registration) stays within the HBM budget;
//   - launch: everything admitted in one scheduling step is planned already
//     and goes out as one batch (products sharing a kernel configuration in
//     one launch) on the least busy of several streams, so requests that
//     arrive while others run are started beside them and their work
//     overlaps on the device;
//   - retirement: each batch ends with an event; when it has completed, its
//     requests are done, their footprint and slots are returned and their
//     latency (submission to completion) is recorded.
// Resident operands: a registered matrix keeps its INT8 digit planes in the
// server; a request whose A (or B) is that matrix skips its digitising pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "mmp_internal.h"

namespace {

using namespace mmp;
using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

struct Operand {
  uint64_t id;
  const double* M;
  int64_t rows, cols, ld;
  uint64_t p;
  int side;  // 0: an A (D planes of rows x kp), 1: a B (D planes of cols x kp)
  int digits;
  int64_t kp;
  int8_t* planes;
  size_t bytes;
};

struct Request {
  uint64_t ticket;
  mmp_job job;
  mmp_plan_t plan;
  size_t footprint;
  double t_submit = 0, t_start = 0, t_done = 0;
  int status = MMP_OK;
  int state = 0;  // 0 queued, 1 running, 2 done
  const Operand* res_a = nullptr;
  const Operand* res_b = nullptr;
  int solo_splits = 1;  // split-K when launched alone (the planner's choice)
  hipEvent_t after = nullptr;  // recorded on the caller's stream at submission
};

struct InFlight {
  int stream;
  hipEvent_t ev = nullptr;
  double sim_end = 0;  // dry-run mode: completion time
  std::vector<uint64_t> tickets;
};

}  // namespace

struct mmp_server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  bool dry_run = false;
  bool fail_launches = false;  // testing aid (MMP_SERVER_FAIL_LAUNCHES)
  std::vector<hipStream_t> streams;
  std::vector<int> stream_load;

  std::mutex mu;
  std::condition_variable cv_sched;  // wakes the scheduler
  std::condition_variable cv_done;   // wakes waiters
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<InFlight> inflight;
  std::map<uint64_t, Operand> operands;
  uint64_t next_ticket = 1, next_operand = 1;
  size_t used = 0, peak_used = 0, resident = 0;
  int slots_used = 0;
  mmp_server_stats_t stats{};
  bool stop = false;
  std::thread th;

  // ---------------------------------------------------------------- helpers
  const Operand* find_resident(const double* M, int64_t rows, int64_t cols, int64_t ld, uint64_t p, int side,
                               int digits, int64_t kp) {
    for (auto& kv : operands) {
      const Operand& o = kv.second;
      if (o.M == M && o.rows == rows && o.cols == cols && o.ld == ld && o.p == p && o.side == side &&
          o.digits == digits && o.kp == kp)
        return &o;
    }
    return nullptr;
  }

  // The request's footprint: operands, result and word copies; for the
  // INT8 form exactly the digit planes the launch allocates (resident planes
  // are not counted again), and the k-range residues of a lone launch.
  size_t request_footprint(const Request& r) const {
    const mmp_job& j = r.job;
    size_t fp;
    if (r.plan.form == MMP_FORM_INT8_WORDS) {
      fp = 8 * ((size_t)(j.m * j.k) + (size_t)(j.k * j.n) + (size_t)(j.m * j.n));
      fp += int8_planes_bytes(r.plan.digits_a, j.m, j.n, j.k, r.res_a != nullptr, r.res_b != nullptr);
    } else {
      mmp_plan_t pl = r.plan;
      fp = mmp_footprint(&j, &pl);
    }
    if (r.solo_splits > 1) fp += 8 * (size_t)r.solo_splits * (size_t)(j.m * j.n);  // k-range residues
    return fp;
  }

  // ---------------------------------------------------------------- scheduler
  // Launches one admitted batch; returns true when the launch failed and
  // its requests were completed with the error (waiters must be woken).
  bool launch_locked(std::vector<uint64_t>& batch) {
    // least busy stream
    int s = (int)(std::min_element(stream_load.begin(), stream_load.end()) - stream_load.begin());
    InFlight f;
    f.stream = s;
    f.tickets = batch;
    const double t0 = now_s();
    double est = 0;
    for (uint64_t t : batch) {
      Request& r = reqs[t];
      r.state = 1;
      r.t_start = t0;
      est += r.plan.est_seconds;
    }
    stats.launches += 1;
    stats.max_batch = std::max<int64_t>(stats.max_batch, (int64_t)batch.size());
    if (fail_launches) {
      for (uint64_t t : batch) finish_locked(reqs[t], MMP_ENOMEM, now_s());
      return true;
    }
    if (dry_run) {
      // no device work: the batch "runs" for the planner's estimate after
      // whatever is already queued on its stream
      double start = t0;
      for (auto& g : inflight)
        if (g.stream == s) start = std::max(start, g.sim_end);
      f.sim_end = start + est;
    } else {
      int err = run_requests_locked(batch, streams[s], inflight.empty());
      if (!err) err = (int)hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
      if (!err) err = (int)hipEventRecord(f.ev, streams[s]);
      if (err) {
        // part of the batch may be enqueued already: let it drain before
        // its buffers and footprint are released
        (void)hipStreamSynchronize(streams[s]);
        const int st = err < 0 ? err : hip_status(err);
        for (uint64_t t : batch) finish_locked(reqs[t], st, now_s());
        if (f.ev) (void)hipEventDestroy(f.ev);
        return true;
      }
    }
    stream_load[s] += 1;
    inflight.push_back(f);
    stats.max_inflight = std::max<int64_t>(stats.max_inflight, (int64_t)inflight.size());
    int64_t running = 0;
    for (auto& g : inflight) running += (int64_t)g.tickets.size();
    stats.max_running = std::max<int64_t>(stats.max_running, running);
    return false;
  }

  // Enqueues the batch on stream s; returns a hipError_t (> 0) or a
  // negative mmp_status.
  int run_requests_locked(const std::vector<uint64_t>& batch, hipStream_t s, bool idle) {
    // FP64-word products grouped by kernel configuration; INT8 products
    // with their planes in one stream-ordered workspace.  Requests that run
    // beside others fill the chip together and each runs whole; a request
    // launched alone on an idle device takes the planner's split-K (a narrow
    // product's few output tiles spread over the CUs by k-range), its
    // residues per k-range after its planes in the workspace.
    std::map<std::tuple<int, int, int, int>, std::vector<Fp64Args>> f64;
    std::map<int, std::vector<Int8Args>> i8;
    const bool solo = idle && batch.size() == 1;
    size_t ws = 0;
    std::vector<size_t> offs, part_off;
    std::vector<int> splits;
    for (uint64_t t : batch) {
      Request& r = reqs[t];
      const mmp_job& j = r.job;
      offs.push_back(ws);
      part_off.push_back(0);
      splits.push_back(1);
      if (j.m == 0 || j.n == 0 || j.k == 0) continue;
      size_t need = 0;
      if (r.plan.form == MMP_FORM_INT8_WORDS)
        need = int8_planes_bytes(r.plan.digits_a, j.m, j.n, j.k, r.res_a != nullptr, r.res_b != nullptr);
      if (solo && r.solo_splits > 1) {
        splits.back() = r.solo_splits;
        part_off.back() = need;
        need += 8 * (size_t)r.solo_splits * (size_t)j.m * (size_t)j.n;
      }
      ws += (need + 255) / 256 * 256;
    }
    // the callers' production of A, B and C comes first (mmp_submit_after)
    for (uint64_t t : batch)
      if (reqs[t].after)
        if (int e = (int)hipStreamWaitEvent(s, reqs[t].after, 0)) return e;
    void* work = nullptr;
    bool owned = false;
    if (int st = acquire_workspace(ws, nullptr, s, &work, &owned)) return st;
    int err = 0;
    for (size_t i = 0; i < batch.size() && !err; i++) {
      Request& r = reqs[batch[i]];
      const mmp_job& j = r.job;
      if (j.m == 0 || j.n == 0) continue;
      if (j.k == 0) {
        err = launch_zero_fill(j.C, j.m, j.n, j.ldc, s);
        continue;
      }
      double* partial = splits[i] > 1 ? (double*)((char*)work + offs[i] + part_off[i]) : nullptr;
      if (r.plan.form == MMP_FORM_FP64_WORDS) {
        Fp64Args a = make_fp64_args(r.plan, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc);
        a.splits = splits[i];
        a.partial = partial;
        f64[std::make_tuple(r.plan.u, r.plan.v, r.plan.tile, fp64_class(r.plan.slots, r.plan.kblock, r.plan.lazy != 0))].push_back(a);
      } else {
        Int8Args g = make_int8_args(r.plan, j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc,
                                    (int8_t*)work + offs[i]);
        g.resident_a = r.res_a ? r.res_a->planes : nullptr;
        g.resident_b = r.res_b ? r.res_b->planes : nullptr;
        g.splits = splits[i];
        g.partial = partial;
        err = launch_int8_digitize(r.plan.digits_a, g, s);
        i8[r.plan.digits_a].push_back(g);
      }
    }
    for (auto& kv : f64) {
      for (size_t c = 0; c < kv.second.size() && !err; c += kMaxBatch) {
        Fp64Batch b;
        std::memset(&b, 0, sizeof(b));
        b.njobs = (int)std::min<size_t>(kMaxBatch, kv.second.size() - c);
        for (int t = 0; t < b.njobs; t++) b.job[t] = kv.second[c + t];
        err = launch_fp64_words(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), b, s);
      }
    }
    for (auto& kv : i8)
      for (size_t c = 0; c < kv.second.size() && !err; c += kMaxBatch)
        err = launch_int8_gemm(kv.first, kv.second.data() + c, (int)std::min<size_t>(kMaxBatch, kv.second.size() - c), s);
    for (size_t i = 0; i < batch.size() && !err; i++) {
      if (splits[i] < 2) continue;
      const mmp_job& j = reqs[batch[i]].job;
      err = launch_splitk_reduce((const double*)((char*)work + offs[i] + part_off[i]), splits[i], j.m, j.n,
                                 (double)j.p, j.C, j.ldc, s);
    }
    const int st2 = release_workspace(work, owned, s);
    if (err) return err;
    return st2;
  }

  void finish_locked(Request& r, int status, double t) {
    if (r.state == 2) return;
    if (r.state == 1) {
      used -= r.footprint;
      slots_used -= 1;
    }
    if (r.after) {  // its wait was enqueued before the batch's work, which has completed
      (void)hipEventDestroy(r.after);
      r.after = nullptr;
    }
    r.state = 2;
    r.status = status;
    r.t_done = t;
    stats.completed += 1;
    if (status != MMP_OK) stats.failed += 1;
  }

  bool retire_locked() {
    bool any = false;
    const double t = now_s();
    for (size_t i = 0; i < inflight.size();) {
      InFlight& f = inflight[i];
      bool done;
      int st = MMP_OK;
      if (dry_run) {
        done = t >= f.sim_end;
      } else {
        hipError_t q = hipEventQuery(f.ev);
        done = q != hipErrorNotReady;
        if (done && q != hipSuccess) st = hip_status((int)q);
      }
      if (!done) {
        i++;
        continue;
      }
      for (uint64_t tk : f.tickets) finish_locked(reqs[tk], st, t);
      if (f.ev) (void)hipEventDestroy(f.ev);
      stream_load[f.stream] -= 1;
      inflight.erase(inflight.begin() + i);
      any = true;
    }
    return any;
  }

  bool admit_locked(std::vector<uint64_t>& batch) {
    while (!queue.empty()) {
      Request& r = reqs[queue.front()];
      if (slots_used + 1 > max_slots || used + r.footprint > budget) break;
      used += r.footprint;
      peak_used = std::max(peak_used, used);
      slots_used += 1;
      batch.push_back(r.ticket);
      queue.pop_front();
    }
    return !batch.empty();
  }

  void loop() {
    if (!dry_run) (void)hipSetDevice(device);
    // This thread's timed waits poll in-flight batches every few
    // microseconds; the kernel's default 50 us timer slack would stretch each
    // of them (and every request's latency) by that much.
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      bool finished = retire_locked();
      std::vector<uint64_t> batch;
      if (admit_locked(batch) && launch_locked(batch)) finished = true;
      if (finished) cv_done.notify_all();
      if (stop && queue.empty() && inflight.empty()) break;
      if (inflight.empty() && queue.empty()) {
        cv_sched.wait(lk, [&] { return stop || !queue.empty(); });
      } else {
        // poll in-flight batches; new submissions wake the loop early
        cv_sched.wait_for(lk, std::chrono::microseconds(10));
      }
    }
    cv_done.notify_all();
  }
};

extern "C" {

int mmp_server_create(mmp_server** out, int device, size_t hbm_budget, int max_slots, int flags) {
  try {
    if (!out || max_slots < 1 || hbm_budget == 0 || (flags & ~(MMP_SERVER_DRY_RUN | MMP_SERVER_FAIL_LAUNCHES)))
      return MMP_EINVAL;
    *out = nullptr;
    auto* s = new mmp_server();
    s->device = device;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->dry_run = (flags & MMP_SERVER_DRY_RUN) != 0;
    s->fail_launches = (flags & MMP_SERVER_FAIL_LAUNCHES) != 0;
    const int nstreams = 4;
    s->stream_load.assign(nstreams, 0);
    if (!s->dry_run) {
      int e = (int)hipSetDevice(device);
      for (int i = 0; i < nstreams && !e; i++) {
        hipStream_t st = nullptr;
        e = (int)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);  // default priority
        if (!e) s->streams.push_back(st);
      }
      if (e) {
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        delete s;
        return hip_status(e);
      }
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return MMP_OK;
  } catch (...) {
    return MMP_ENOMEM;
  }
}

int mmp_server_destroy(mmp_server* s) {
  if (!s) return MMP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_all();
  if (s->th.joinable()) s->th.join();  // drains queued and running work first
  for (auto& kv : s->operands) (void)hipFree(kv.second.planes);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return MMP_OK;
}

int mmp_register_operand(mmp_server* s, const double* M, int64_t rows, int64_t cols, int64_t ld, uint64_t p,
                         int side, uint64_t* handle) {
  try {
    if (!s || !handle || !M || rows <= 0 || cols <= 0 || ld < cols || (side != 0 && side != 1)) return MMP_EINVAL;
    if (p < 5 || p >= kPMax) return MMP_EINVAL;
    if (s->dry_run) return MMP_EINVAL;
    Operand o;
    o.M = M;
    o.rows = rows;
    o.cols = cols;
    o.ld = ld;
    o.p = p;
    o.side = side;
    o.digits = digits_for(p);
    const int64_t kdim = side == 0 ? cols : rows;  // the inner dimension
    const int64_t outer = side == 0 ? rows : cols;
    o.kp = (kdim + 63) / 64 * 64;
    o.bytes = digit_planes_bytes(o.digits, outer, o.kp);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->used + o.bytes > s->budget) return MMP_ENOMEM;
    if (int e = (int)hipSetDevice(s->device)) return hip_status(e);
    if (int e = (int)hipMalloc(&o.planes, o.bytes)) return hip_status(e);
    hipStream_t st = s->streams[0];
    int e = launch_int8_digitize_side(o.digits, side, M, rows, cols, ld, o.kp, p, o.planes, st);
    if (!e) e = (int)hipStreamSynchronize(st);
    if (e) {
      (void)hipFree(o.planes);
      return hip_status(e);
    }
    o.id = s->next_operand++;
    s->used += o.bytes;
    s->resident += o.bytes;
    s->peak_used = std::max(s->peak_used, s->used);
    s->operands[o.id] = o;
    *handle = o.id;
    return MMP_OK;
  } catch (...) {
    return MMP_ENOMEM;
  }
}

int mmp_unregister_operand(mmp_server* s, uint64_t handle) {
  if (!s) return MMP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->operands.find(handle);
  if (it == s->operands.end()) return MMP_ENOTFOUND;
  // wait until no queued or running request uses it
  s->cv_done.wait(lk, [&] {
    for (auto& kv : s->reqs)
      if (kv.second.state != 2 && (kv.second.res_a == &it->second || kv.second.res_b == &it->second)) return false;
    return true;
  });
  (void)hipFree(it->second.planes);
  s->used -= it->second.bytes;
  s->resident -= it->second.bytes;
  s->operands.erase(it);
  return MMP_OK;
}

static int submit_impl(mmp_server* s, const mmp_job* job, int flags, bool ordered, void* stream,
                       uint64_t* ticket) {
  hipEvent_t after = nullptr;
  try {
    if (!s || !job || !ticket || (flags & ~MMP_SUBMIT_NOQUEUE)) return MMP_EINVAL;
    const mmp_job& j = *job;
    if (int st = check_product_args(j.m, j.n, j.k, j.A, j.lda, j.B, j.ldb, j.C, j.ldc)) return st;
    Request r;
    r.job = j;
    mmp_opts o1;
    std::memset(&o1, 0, sizeof(o1));
    o1.splits = 1;  // requests run whole; concurrency comes from the mix
    if (int st = mmp::plan(j.p, j.u, j.v, j.m, j.n, j.k, &o1, &r.plan)) return st;
    if (!fp64_ld_ok(r.plan, j.lda, j.ldb)) {  // an AUTO request takes the INT8 form instead
      if (j.u != 0) return MMP_EINVAL;
      o1.form = MMP_FORM_INT8_WORDS;
      if (int st = mmp::plan(j.p, 0, 0, j.m, j.n, j.k, &o1, &r.plan)) return st;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    // An AUTO request with an operand whose digit planes are resident takes
    // the INT8 form: the planner's estimate charges for digitising both
    // operands, which a resident operand no longer needs.
    if (r.plan.form == MMP_FORM_FP64_WORDS && j.u == 0 && j.m > 0 && j.n > 0 && j.k > 0) {
      mmp_opts o8 = o1;
      o8.form = MMP_FORM_INT8_WORDS;
      mmp_plan_t p8;
      if (mmp::plan(j.p, 0, 0, j.m, j.n, j.k, &o8, &p8) == MMP_OK) {
        const int64_t kp = (j.k + 63) / 64 * 64;
        if (s->find_resident(j.A, j.m, j.k, j.lda, j.p, 0, p8.digits_a, kp) ||
            s->find_resident(j.B, j.k, j.n, j.ldb, j.p, 1, p8.digits_b, kp))
          r.plan = p8;
      }
    }
    if (r.plan.form == MMP_FORM_INT8_WORDS) {
      const int64_t kp = (j.k + 63) / 64 * 64;
      r.res_a = s->find_resident(j.A, j.m, j.k, j.lda, j.p, 0, r.plan.digits_a, kp);
      r.res_b = s->find_resident(j.B, j.k, j.n, j.ldb, j.p, 1, r.plan.digits_b, kp);
    }
    r.solo_splits = default_splits(r.plan, j.m, j.n, j.k);
    r.footprint = s->request_footprint(r);
    if (r.footprint > s->budget - s->resident) {
      s->stats.rejected += 1;
      return MMP_ENOMEM;  // can never be admitted
    }
    if ((flags & MMP_SUBMIT_NOQUEUE) &&
        (!s->queue.empty() || s->slots_used + 1 > s->max_slots || s->used + r.footprint > s->budget)) {
      s->stats.rejected += 1;
      return MMP_EBUSY;
    }
    if (ordered && !s->dry_run) {  // a NULL stream is the null stream
      if (int e = (int)hipEventCreateWithFlags(&after, hipEventDisableTiming)) return hip_status(e);
      if (int e = (int)hipEventRecord(after, (hipStream_t)stream)) {
        (void)hipEventDestroy(after);
        return hip_status(e);
      }
      r.after = after;
    }
    r.ticket = s->next_ticket++;
    r.t_submit = now_s();
    s->stats.submitted += 1;
    const uint64_t t = r.ticket;
    s->reqs.emplace(t, r);
    s->queue.push_back(t);
    *ticket = t;
    s->cv_sched.notify_all();
    return MMP_OK;
  } catch (...) {
    if (after) (void)hipEventDestroy(after);
    return MMP_ENOMEM;
  }
}

int mmp_submit(mmp_server* s, const mmp_job* job, int flags, uint64_t* ticket) {
  return submit_impl(s, job, flags, false, nullptr, ticket);
}

int mmp_submit_after(mmp_server* s, const mmp_job* job, int flags, void* stream, uint64_t* ticket) {
  return submit_impl(s, job, flags, true, stream, ticket);
}

static int report(mmp_server* s, std::unordered_map<uint64_t, Request>::iterator it, int* status, double* latency) {
  if (status) *status = it->second.status;
  if (latency) *latency = it->second.t_done - it->second.t_submit;
  s->reqs.erase(it);  // a reported ticket is forgotten
  return MMP_OK;
}

int mmp_poll(mmp_server* s, uint64_t ticket, int* done, int* status, double* latency_s) {
  if (!s || !done) return MMP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MMP_ENOTFOUND;
  *done = it->second.state == 2;
  if (!*done) return MMP_OK;
  return report(s, it, status, latency_s);
}

int mmp_wait(mmp_server* s, uint64_t ticket, double timeout_s, int* status, double* latency_s) {
  if (!s) return MMP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MMP_ENOTFOUND;
  auto pred = [&] {
    auto f = s->reqs.find(ticket);
    return f == s->reqs.end() || f->second.state == 2;
  };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return MMP_ETIMEOUT;
  }
  auto f = s->reqs.find(ticket);
  if (f == s->reqs.end()) return MMP_ENOTFOUND;  // reported to another caller meanwhile
  return report(s, f, status, latency_s);
}

int mmp_server_stats(mmp_server* s, mmp_server_stats_t* out) {
  if (!s || !out) return MMP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = (int64_t)s->queue.size();
  int64_t running = 0;
  for (auto& f : s->inflight) running += (int64_t)f.tickets.size();
  out->running = running;
  out->used_bytes = s->used;
  out->peak_used_bytes = s->peak_used;
  out->resident_bytes = s->resident;
  return MMP_OK;
}

}  // extern "C"
