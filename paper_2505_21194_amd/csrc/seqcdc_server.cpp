// Serving: a dedup-ingest request loop with continuous batching.
//
// Requests reference device-resident bytes.  A scheduler thread admits queued
// requests while the device memory they need (input bytes, mark bitmaps,
// segment lists and cut output) fits the budget and a ring slot is free,
// groups them (up to max_batch) into one batched pass on a free stream, and
// keeps admitting while earlier passes run: passes on different streams
// overlap on the GPU.  When a pass's event completes, each request's cuts are
// published to host memory with its latency.  A request that has waited longer
// than all others and does not fit blocks further admission until it does, so
// large requests are not starved by a stream of small ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

constexpr u32 kServerWaves = 8;  // chain waves per CU of each serving pass

using Clock = std::chrono::steady_clock;

static double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  u64 ticket;
  const void* data;
  u64 n;
  u32 pidx;
  u64 cost;
  Clock::time_point t_submit, t_admit, t_done;
  int status = SEQCDC_EAGAIN;
  std::vector<u64> cuts;
};

struct Pass {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Plan plan;
  DevBuf d_cuts, d_counts;
  HostBuf h_cuts, h_counts;
  std::vector<Request*> reqs;
  std::vector<u64> offs;
  u64 bytes = 0;
};

struct Server {
  seqcdc_server_config cfg;
  std::vector<seqcdc_params> params;
  u64 min_min = 0;
  std::vector<Pass*> passes;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Request*> queue;
  std::map<u64, Request*> all;
  u64 next_ticket = 1;
  u64 bytes_inflight = 0, reqs_inflight = 0;
  u64 stat_admitted = 0, stat_passes = 0, stat_peak_bytes = 0, stat_peak_reqs = 0;
  bool stop = false;
  std::thread th;
  int thread_err = SEQCDC_OK;

  u64 cost_of(u64 n, const seqcdc_params& p) const {
    // input + EO16 bitmaps + per-segment lists + cut output (device) + fixed overhead
    return n + 16 * ((n + 63) / 64) + 16 * (n / p.min_size + 2) + (64 << 10);
  }
};

static int launch_pass(Server* s, Pass* ps) {
  const u32 nf = (u32)ps->reqs.size();
  std::vector<seqcdc_file> files(nf);
  ps->offs.assign(nf + 1, 0);
  for (u32 i = 0; i < nf; i++) {
    Request* r = ps->reqs[i];
    files[i] = seqcdc_file{r->data, r->n, r->pidx, 0};
    ps->offs[i + 1] = ps->offs[i] + std::max<u64>(max_cuts(r->n, &s->params[r->pidx]), 1);
  }
  const u64 total = ps->offs[nf];
  int rc;
  if ((rc = ps->d_cuts.reserve(total * 8))) return rc;
  if ((rc = ps->d_counts.reserve(nf * 8))) return rc;
  if ((rc = ps->h_cuts.reserve(total * 8))) return rc;
  if ((rc = ps->h_counts.reserve(nf * 8))) return rc;
  rc = chunk_batch(&ps->plan, files.data(), nf, s->params.data(), (u32)s->params.size(), (u64*)ps->d_cuts.p,
                   ps->offs.data(), (u64*)ps->d_counts.p, ps->stream);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(ps->h_counts.p, ps->d_counts.p, nf * 8, hipMemcpyDeviceToHost, ps->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ps->h_cuts.p, ps->d_cuts.p, total * 8, hipMemcpyDeviceToHost, ps->stream);
  if (e == hipSuccess) e = hipEventRecord(ps->done, ps->stream);
  if (e != hipSuccess) return hip_fail(e, "serving pass");
  ps->busy = true;
  return SEQCDC_OK;
}

static void finish_pass(Server* s, Pass* ps, int status) {
  const u64* counts = (const u64*)ps->h_counts.p;
  const u64* cuts = (const u64*)ps->h_cuts.p;
  std::lock_guard<std::mutex> g(s->mu);
  const auto now = Clock::now();
  for (size_t i = 0; i < ps->reqs.size(); i++) {
    Request* r = ps->reqs[i];
    if (status == SEQCDC_OK) {
      r->cuts.assign(cuts + ps->offs[i], cuts + ps->offs[i] + counts[i]);
      r->status = SEQCDC_OK;
    } else {
      r->status = status;
    }
    r->t_done = now;
    s->bytes_inflight -= r->cost;
    s->reqs_inflight--;
  }
  ps->plan.pending = false;
  ps->plan.upload_pending = false;
  ps->reqs.clear();
  ps->busy = false;
  s->cv_done.notify_all();
}

static void scheduler(Server* s) {
  if (hipSetDevice(s->cfg.device) != hipSuccess) {
    s->thread_err = SEQCDC_EHIP;
    return;
  }
  for (;;) {
    // 1. retire finished passes
    bool any_busy = false;
    Pass* free_pass = nullptr;
    for (Pass* ps : s->passes) {
      if (ps->busy) {
        hipError_t q = hipEventQuery(ps->done);
        if (q == hipSuccess) finish_pass(s, ps, SEQCDC_OK);
        else if (q != hipErrorNotReady) finish_pass(s, ps, SEQCDC_EHIP);
      }
      if (ps->busy) any_busy = true;
      else if (!free_pass) free_pass = ps;
    }
    // 2. admit a group of queued requests into the free pass
    std::vector<Request*> group;
    u64 group_bytes = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop && s->queue.empty() && !any_busy) return;
      if (free_pass) {
        for (auto it = s->queue.begin(); it != s->queue.end() && group.size() < s->cfg.max_batch;) {
          Request* r = *it;
          const bool fits = s->bytes_inflight + group_bytes + r->cost <= s->cfg.budget_bytes &&
                            s->reqs_inflight + group.size() < s->cfg.ring_slots;
          if (fits) {
            group.push_back(r);
            group_bytes += r->cost;
            it = s->queue.erase(it);
          } else if (it == s->queue.begin()) {
            break;  // the oldest request waits for room; nothing may overtake it
          } else {
            ++it;
          }
        }
      }
      if (group.empty()) {
        // 3. idle: poll the GPU briefly while passes run, else sleep until a submission
        if (any_busy) s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else s->cv_sched.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
      const auto now = Clock::now();
      for (Request* r : group) r->t_admit = now;
      s->bytes_inflight += group_bytes;
      s->reqs_inflight += group.size();
      s->stat_admitted += group.size();
      s->stat_passes++;
      s->stat_peak_bytes = std::max(s->stat_peak_bytes, s->bytes_inflight);
      s->stat_peak_reqs = std::max(s->stat_peak_reqs, s->reqs_inflight);
    }
    free_pass->reqs = group;
    free_pass->bytes = group_bytes;
    int rc = launch_pass(s, free_pass);
    if (rc) finish_pass(s, free_pass, rc);
  }
}

}  // namespace seqcdc

using namespace seqcdc;

extern "C" {

int seqcdc_server_create(const seqcdc_server_config* cfg, seqcdc_server** out) {
  if (!cfg || !out) return fail(SEQCDC_EINVAL, "NULL argument");
  if (cfg->nparams == 0 || !cfg->params) return fail(SEQCDC_EINVAL, "at least one parameter set is required");
  if (cfg->streams == 0 || cfg->streams > 8) return fail(SEQCDC_EINVAL, "streams must be in [1, 8]");
  if (cfg->ring_slots == 0 || cfg->max_batch == 0) return fail(SEQCDC_EINVAL, "ring_slots and max_batch must be > 0");
  for (u32 i = 0; i < cfg->nparams; i++) {
    int rc = validate(&cfg->params[i]);
    if (rc) return rc;
  }
  Server* s = new (std::nothrow) Server();
  if (!s) return fail(SEQCDC_ENOMEM, "server allocation failed");
  s->cfg = *cfg;
  s->params.assign(cfg->params, cfg->params + cfg->nparams);
  s->cfg.params = s->params.data();
  int dev = cfg->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
    delete s;
    return fail(SEQCDC_EHIP, "hipGetDevice failed");
  }
  s->cfg.device = dev;
  for (u32 i = 0; i < cfg->streams; i++) {
    Pass* ps = new Pass();
    int rc = plan_init(&ps->plan, dev);
    // Passes are batches of many requests, mostly small, several in flight:
    // the marked resolve, no overlapped groups, and a fixed chain occupancy,
    // so that one pass's persistent chain kernels leave room (LDS, wave
    // slots) for the others'.
    ps->plan.mode = 0;
    ps->plan.overlap = 1;
    ps->plan.waves_override = kServerWaves;
    hipError_t e = hipSuccess;
    if (!rc) e = hipStreamCreateWithFlags(&ps->stream, hipStreamNonBlocking);
    if (!rc && e == hipSuccess) e = hipEventCreateWithFlags(&ps->done, hipEventDisableTiming);
    if (rc || e != hipSuccess) {
      delete ps;
      for (Pass* p : s->passes) {
        plan_free(&p->plan);
        delete p;
      }
      delete s;
      return rc ? rc : hip_fail(e, "server stream");
    }
    s->passes.push_back(ps);
  }
  s->th = std::thread(scheduler, s);
  *out = (seqcdc_server*)s;
  return SEQCDC_OK;
}

int seqcdc_server_submit(seqcdc_server* sv, const void* d_data, uint64_t n, uint32_t pidx, uint64_t* ticket) {
  Server* s = (Server*)sv;
  if (!s || !ticket) return fail(SEQCDC_EINVAL, "NULL argument");
  if (pidx >= s->params.size()) return fail(SEQCDC_EINVAL, "params_index out of range");
  if (n && !d_data) return fail(SEQCDC_EINVAL, "NULL data");
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(SEQCDC_ENOMEM, "request allocation failed");
  r->data = d_data;
  r->n = n;
  r->pidx = pidx;
  r->cost = s->cost_of(n, s->params[pidx]);
  r->t_submit = Clock::now();
  if (r->cost > s->cfg.budget_bytes) {
    delete r;
    return fail(SEQCDC_EBUDGET, "request needs %llu bytes, budget is %llu", (unsigned long long)s->cost_of(n, s->params[pidx]),
                (unsigned long long)s->cfg.budget_bytes);
  }
  std::lock_guard<std::mutex> g(s->mu);
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->all[r->ticket] = r;
  if (n == 0) {
    r->status = SEQCDC_OK;
    r->t_admit = r->t_done = r->t_submit;
    s->cv_done.notify_all();
    return SEQCDC_OK;
  }
  s->queue.push_back(r);
  s->cv_sched.notify_one();
  return SEQCDC_OK;
}

static void fill(const Request* r, seqcdc_result* out) {
  out->status = r->status;
  out->reserved = 0;
  out->count = r->status == SEQCDC_OK ? r->cuts.size() : 0;
  out->cuts = r->status == SEQCDC_OK ? r->cuts.data() : nullptr;
  out->latency_ms = r->status == SEQCDC_EAGAIN ? 0.0 : ms_between(r->t_submit, r->t_done);
  out->queue_ms = r->status == SEQCDC_EAGAIN ? 0.0 : ms_between(r->t_submit, r->t_admit);
}

int seqcdc_server_poll(seqcdc_server* sv, uint64_t ticket, seqcdc_result* out) {
  Server* s = (Server*)sv;
  if (!s || !out) return fail(SEQCDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(SEQCDC_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
  fill(it->second, out);
  return it->second->status == SEQCDC_EAGAIN ? SEQCDC_EAGAIN : it->second->status;
}

int seqcdc_server_wait(seqcdc_server* sv, uint64_t ticket, double timeout_ms, seqcdc_result* out) {
  Server* s = (Server*)sv;
  if (!s || !out) return fail(SEQCDC_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(SEQCDC_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  auto pred = [&] { return r->status != SEQCDC_EAGAIN; };
  if (timeout_ms < 0) s->cv_done.wait(lk, pred);
  else s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred);
  fill(r, out);
  return r->status;
}

int seqcdc_server_release(seqcdc_server* sv, uint64_t ticket) {
  Server* s = (Server*)sv;
  if (!s) return fail(SEQCDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(SEQCDC_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->status == SEQCDC_EAGAIN) return fail(SEQCDC_EAGAIN, "request still running");
  delete it->second;
  s->all.erase(it);
  return SEQCDC_OK;
}

int seqcdc_server_stats(seqcdc_server* sv, uint64_t* admitted, uint64_t* passes, uint64_t* peak_bytes,
                        uint64_t* peak_inflight) {
  Server* s = (Server*)sv;
  if (!s) return fail(SEQCDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  if (admitted) *admitted = s->stat_admitted;
  if (passes) *passes = s->stat_passes;
  if (peak_bytes) *peak_bytes = s->stat_peak_bytes;
  if (peak_inflight) *peak_inflight = s->stat_peak_reqs;
  return SEQCDC_OK;
}

int seqcdc_server_destroy(seqcdc_server* sv) {
  Server* s = (Server*)sv;
  if (!s) return SEQCDC_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_sched.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (Pass* ps : s->passes) {
    if (ps->busy) (void)hipEventSynchronize(ps->done);
    plan_free(&ps->plan);
    ps->d_cuts.release();
    ps->d_counts.release();
    ps->h_cuts.release();
    ps->h_counts.release();
    if (ps->done) (void)hipEventDestroy(ps->done);
    if (ps->stream) (void)hipStreamDestroy(ps->stream);
    delete ps;
  }
  for (auto& kv : s->all) delete kv.second;
  for (Request* r : s->queue)
    if (!s->all.count(r->ticket)) delete r;
  delete s;
  return SEQCDC_OK;
}

}  // extern "C"
