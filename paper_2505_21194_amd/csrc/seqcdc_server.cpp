// Serving: a dedup-ingest request loop with continuous batching.
//
// Requests reference device-resident bytes.  The budget is split evenly
// between the passes (one per stream).  At creation each pass reserves, once,
// the workspace (mark bitmaps, segment lists, continuation buffers, tables,
// cut output on the device and in pinned host memory) for the largest group
// of requests its share can hold: its input capacity plus that workspace fit
// the share.  A scheduler thread admits queued requests into a free pass while
// their bytes fit its capacity and a ring slot is free (up to max_batch per
// pass) and launches the group as one batched pass on the pass's stream; it
// keeps admitting while earlier passes run, so passes on different streams
// overlap on the GPU, and nothing is allocated or freed on this path.  When a
// pass's event completes, each request's cuts are published to host memory
// with its latency.  The oldest queued request is never overtaken: it waits
// for a free pass, which can always hold it, so large requests are not starved
// by a stream of small ones.
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

constexpr size_t kTimelineKeep = 4096;  // pass records kept for seqcdc_server_timeline

struct Pass {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;  // timing events around the pass's work on its stream
  seqcdc_pass_record rec{};                    // the pass in flight
  Clock::time_point t_admit, t_enqueued;
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
  std::vector<Pass*> passes;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::deque<Request*> queue;
  std::map<u64, Request*> all;
  u64 next_ticket = 1;
  u64 bytes_inflight = 0, reqs_inflight = 0;
  u64 stat_admitted = 0, stat_passes = 0, stat_peak_bytes = 0, stat_peak_reqs = 0;
  std::deque<seqcdc_pass_record> timeline;  // the latest passes, oldest first
  bool stop = false;
  std::thread th;
  int thread_err = SEQCDC_OK;

  u64 pass_cap = 0;   // input bytes one pass can hold (its workspace is reserved for them)
  u64 workspace = 0;  // device and pinned bytes all passes reserved at creation
  u64 min_min = ~0ull;

  u64 cost_of(u64 n, const seqcdc_params& p) const {
    (void)p;
    return n;  // input bytes; the workspace is reserved per pass
  }
};

static int launch_pass(Server* s, Pass* ps) {
  const auto t0 = Clock::now();
  const u64 reallocs0 = realloc_count();
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
  hipError_t e0 = hipEventRecord(ps->start, ps->stream);
  if (e0 != hipSuccess) return hip_fail(e0, "serving pass");
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
  ps->t_enqueued = Clock::now();
  ps->rec.requests = nf;
  ps->rec.bytes = 0;
  for (Request* r : ps->reqs) ps->rec.bytes += r->n;
  ps->rec.grew = (u32)(realloc_count() - reallocs0);
  ps->rec.wait_ms = ms_between(ps->t_admit, t0);
  ps->rec.layout_ms = ms_between(t0, ps->t_enqueued);
  return SEQCDC_OK;
}

static void finish_pass(Server* s, Pass* ps, int status) {
  const u64* counts = (const u64*)ps->h_counts.p;
  const u64* cuts = (const u64*)ps->h_cuts.p;
  float gpu_ms = 0;
  if (status == SEQCDC_OK && hipEventElapsedTime(&gpu_ms, ps->start, ps->done) != hipSuccess) gpu_ms = -1;
  std::lock_guard<std::mutex> g(s->mu);
  const auto now = Clock::now();
  if (status == SEQCDC_OK) {
    ps->rec.gpu_ms = gpu_ms;
    ps->rec.retire_ms = ms_between(ps->t_enqueued, now);
    s->timeline.push_back(ps->rec);
    if (s->timeline.size() > kTimelineKeep) s->timeline.pop_front();
  }
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
        // With several passes free, each takes an equal share of the queued
        // bytes, so a backlog runs as passes in flight together (one pass's
        // resolve overlaps another's marking) rather than as one large pass.
        u32 nfree = 0;
        for (Pass* ps : s->passes) nfree += ps->busy ? 0u : 1u;
        u64 limit = s->pass_cap;
        if (nfree > 1) {
          u64 queued = 0;
          for (Request* r : s->queue) queued += r->cost;
          limit = std::min<u64>(limit, (queued + nfree - 1) / nfree);
        }
        for (auto it = s->queue.begin(); it != s->queue.end() && group.size() < s->cfg.max_batch;) {
          Request* r = *it;
          const bool room = group.empty() ? r->cost <= s->pass_cap : group_bytes + r->cost <= limit;
          const bool fits = room && s->reqs_inflight + group.size() < s->cfg.ring_slots;
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
      free_pass->t_admit = now;
      s->bytes_inflight += group_bytes;
      s->reqs_inflight += group.size();
      s->stat_admitted += group.size();
      s->stat_passes++;
      s->stat_peak_bytes = std::max(s->stat_peak_bytes, s->bytes_inflight + s->workspace);
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
    if (!rc && e == hipSuccess) e = hipEventCreate(&ps->start);
    if (!rc && e == hipSuccess) e = hipEventCreate(&ps->done);
    if (rc || e != hipSuccess) {
      if (ps->done) (void)hipEventDestroy(ps->done);
      if (ps->start) (void)hipEventDestroy(ps->start);
      if (ps->stream) (void)hipStreamDestroy(ps->stream);
      if (!rc) plan_free(&ps->plan);
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
  // Each pass's share of the budget holds its input capacity plus the
  // workspace reserved for it; shrink the capacity until both fit.
  for (u32 i = 0; i < cfg->nparams; i++) s->min_min = std::min<u64>(s->min_min, cfg->params[i].min_size);
  const u64 share = cfg->budget_bytes / cfg->streams;
  const u32 nb = cfg->max_batch;
  auto need = [&](u64 cap) {
    u64 ws = 0;
    (void)plan_reserve(&s->passes[0]->plan, cap, nb, s->params.data(), cfg->nparams, true, &ws);
    const u64 cuts = (cap / s->min_min + nb) * 8;
    return cap + ws + 2 * (cuts + cuts / 4) + 4 * (nb * 8 + 4096);
  };
  u64 cap = share;
  for (int it = 0; it < 64 && cap > 0 && need(cap) > share; it++)
    cap = (u64)((double)cap * (double)share / (double)need(cap) * 0.985);
  int rc = (cap == 0 || need(cap) > share) ? fail(SEQCDC_EINVAL, "budget too small for %u streams", cfg->streams)
                                           : SEQCDC_OK;
  s->pass_cap = cap;
  const u64 cuts = (cap / s->min_min + nb) * 8;
  for (Pass* ps : s->passes) {
    if (rc) break;
    u64 ws = 0;
    rc = plan_reserve(&ps->plan, cap, nb, s->params.data(), cfg->nparams, false, &ws);
    if (!rc) rc = ps->d_cuts.reserve(cuts);
    if (!rc) rc = ps->h_cuts.reserve(cuts);
    if (!rc) rc = ps->d_counts.reserve(nb * 8);
    if (!rc) rc = ps->h_counts.reserve(nb * 8);
    s->workspace += ws + ps->d_cuts.cap + ps->h_cuts.cap + ps->d_counts.cap + ps->h_counts.cap;
  }
  if (rc) {
    for (Pass* p : s->passes) {
      plan_free(&p->plan);
      p->d_cuts.release();
      p->h_cuts.release();
      p->d_counts.release();
      p->h_counts.release();
      if (p->done) (void)hipEventDestroy(p->done);
      if (p->start) (void)hipEventDestroy(p->start);
      if (p->stream) (void)hipStreamDestroy(p->stream);
      delete p;
    }
    delete s;
    return rc;
  }
  s->th = std::thread(scheduler, s);
  *out = (seqcdc_server*)s;
  return SEQCDC_OK;
}

int seqcdc_server_submit_many(seqcdc_server* sv, const seqcdc_file* reqs, uint32_t n, const double* at_ms,
                              uint64_t* tickets, double* submitted_ms) {
  Server* s = (Server*)sv;
  if (!s || (n && (!reqs || !tickets))) return fail(SEQCDC_EINVAL, "NULL argument");
  for (uint32_t i = 0; i < n; i++) {
    const seqcdc_file& f = reqs[i];
    if (f.reserved) return fail(SEQCDC_EINVAL, "request %u: reserved must be 0", i);
    if (f.params_index >= s->params.size()) return fail(SEQCDC_EINVAL, "request %u: params_index out of range", i);
    if (f.n && !f.d_data) return fail(SEQCDC_EINVAL, "request %u: NULL data", i);
    if (s->cost_of(f.n, s->params[f.params_index]) > s->pass_cap)
      return fail(SEQCDC_EBUDGET, "request %u is larger than a pass can hold (%llu bytes)", i,
                  (unsigned long long)s->pass_cap);
    if (at_ms && i && at_ms[i] < at_ms[i - 1]) return fail(SEQCDC_EINVAL, "at_ms must not decrease");
  }
  std::vector<Request*> rs(n);
  for (uint32_t i = 0; i < n; i++) {
    rs[i] = new (std::nothrow) Request();
    if (!rs[i]) {
      for (uint32_t j = 0; j < i; j++) delete rs[j];
      return fail(SEQCDC_ENOMEM, "request allocation failed");
    }
    rs[i]->data = reqs[i].d_data;
    rs[i]->n = reqs[i].n;
    rs[i]->pidx = reqs[i].params_index;
    rs[i]->cost = s->cost_of(reqs[i].n, s->params[reqs[i].params_index]);
  }
  const auto t0 = Clock::now();
  uint32_t i = 0;
  while (i < n) {
    // queue every request that is due, under one lock
    const double now_ms = ms_between(t0, Clock::now());
    uint32_t j = i;
    if (!at_ms) j = n;
    else
      while (j < n && at_ms[j] <= now_ms) j++;
    if (j == i) {  // the next arrival is in the future: wait for it (short sleeps, then spin)
      const double ahead = at_ms[i] - now_ms;
      if (ahead > 0.2) std::this_thread::sleep_for(std::chrono::microseconds((long)((ahead - 0.1) * 1000)));
      continue;
    }
    std::lock_guard<std::mutex> g(s->mu);
    const auto t_sub = Clock::now();
    for (uint32_t k = i; k < j; k++) {
      Request* r = rs[k];
      r->t_submit = t_sub;
      r->ticket = s->next_ticket++;
      tickets[k] = r->ticket;
      if (submitted_ms) submitted_ms[k] = ms_between(t0, t_sub);
      s->all[r->ticket] = r;
      if (r->n == 0) {
        r->status = SEQCDC_OK;
        r->t_admit = r->t_done = t_sub;
      } else {
        s->queue.push_back(r);
      }
    }
    s->cv_sched.notify_one();
    s->cv_done.notify_all();
    i = j;
  }
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
  if (r->cost > s->pass_cap) {
    delete r;
    return fail(SEQCDC_EBUDGET, "request of %llu bytes is larger than a pass can hold (%llu bytes of the %llu budget)",
                (unsigned long long)n, (unsigned long long)s->pass_cap, (unsigned long long)s->cfg.budget_bytes);
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

int seqcdc_server_timeline(seqcdc_server* sv, seqcdc_pass_record* out, uint32_t cap, uint32_t* count) {
  Server* s = (Server*)sv;
  if (!s || !count || (!out && cap)) return fail(SEQCDC_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  const size_t n = std::min<size_t>(cap, s->timeline.size());
  const size_t first = s->timeline.size() - n;
  for (size_t i = 0; i < n; i++) out[i] = s->timeline[first + i];
  *count = (uint32_t)n;
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
    if (ps->start) (void)hipEventDestroy(ps->start);
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
