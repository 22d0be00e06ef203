// Autotuner: picks the segment length of speculative resolution, the mark
// span, the waves per CU of the persistent chain kernels and the resolve mode
// (marked or direct) by timing candidates on a device-resident sample.  Every candidate produces the same
// cuts; only speed differs.  A single stream's results go to a process-wide
// cache keyed by (arch, CU count, SeqLength, average class); a batch's results
// become the plan's own settings, since the best settings for many files
// differ from those for one stream of the same parameters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

static int time_config(Plan* pl, const void* d, u64 n, const seqcdc_params* p, u64* d_cuts, u64 cap,
                       hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, double* ms) {
  u64 cnt = 0;
  int rc = chunk_plan(pl, d, n, p, d_cuts, cap, &cnt, st);  // warm-up (and workspace growth)
  if (rc) return rc;
  double best = 1e30;
  for (int r = 0; r < reps; r++) {
    hipError_t e = hipEventRecord(e0, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    rc = chunk_plan(pl, d, n, p, d_cuts, cap, &cnt, st);
    if (rc) return rc;
    e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "hipEvent timing");
    best = std::min(best, (double)t);
  }
  *ms = best;
  return SEQCDC_OK;
}

// Best of `reps` timed batched calls (after one untimed call).
static int time_batch(Plan* pl, const seqcdc_file* files, u32 nfiles, const seqcdc_params* params, u32 nparams,
                      u64* d_cuts, const u64* h_offs, u64* d_counts, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                      int reps, double* ms) {
  int rc = chunk_batch(pl, files, nfiles, params, nparams, d_cuts, h_offs, d_counts, st);
  if (rc) return rc;
  double best = 1e30;
  for (int r = 0; r < reps; r++) {
    hipError_t e = hipEventRecord(e0, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    rc = chunk_batch(pl, files, nfiles, params, nparams, d_cuts, h_offs, d_counts, st);
    if (rc) return rc;
    e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "hipEvent timing");
    best = std::min(best, (double)t);
  }
  *ms = best;
  return SEQCDC_OK;
}

// One timed setting of a search.  The searches time each candidate briefly,
// then time the few fastest again for longer before choosing: a brief trial's
// best call can be a lucky draw.
struct Candidate {
  u64 seg;  // segment multiple of min_size (one stream) or segment length in bytes (a batch)
  u32 span, waves;
  int mode;
  double ms;
};
constexpr int kTrialReps = 3;   // timed calls per candidate in the search
constexpr int kFinalReps = 10;  // timed calls per finalist
constexpr size_t kFinalists = 3;

std::vector<Candidate> finalists(std::vector<Candidate> c) {
  std::sort(c.begin(), c.end(), [](const Candidate& a, const Candidate& b) { return a.ms < b.ms; });
  if (c.size() > kFinalists) c.resize(kFinalists);
  return c;
}

}  // namespace seqcdc

using namespace seqcdc;

extern "C" int seqcdc_autotune(seqcdc_plan* plan, const void* d_sample, uint64_t n, const seqcdc_params* p,
                               double* best_ms, void* stream) {
  if (!plan) return fail(SEQCDC_EINVAL, "plan is NULL");
  int rc = validate(p);
  if (rc) return rc;
  if (!d_sample || n == 0) return fail(SEQCDC_EINVAL, "empty sample");
  Plan* pl = (Plan*)plan;
  hipStream_t st = (hipStream_t)stream;
  const u64 cap = max_cuts(n, p);
  u64* d_cuts = nullptr;
  hipError_t e = hipMalloc((void**)&d_cuts, cap * 8);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);

  const u64 saved_seg = pl->seg_override;
  const u32 saved_span = pl->span_override, saved_waves = pl->waves_override;
  const int saved_mode = pl->mode;
  pl->mode = 0;
  TuneEntry best;
  best.key = plan_key(pl, p);
  best.sample = n;
  best.ms = 1e30;
  std::vector<Candidate> tried;
  auto trial = [&](u64 seg_mult, u32 span, u32 waves) -> int {
    pl->seg_override = seg_mult * p->min_size;
    pl->span_override = span;
    pl->waves_override = waves;
    double ms = 0;
    int r = time_config(pl, d_sample, n, p, d_cuts, cap, st, e0, e1, kTrialReps, &ms);
    if (r) return r;
    tried.push_back(Candidate{seg_mult, span, waves, pl->mode, ms});
    if (ms < best.ms) {
      best.ms = ms;
      best.seg_mult = seg_mult;
      best.span_blocks = span;
      best.waves_per_cu = waves;
      best.mode = pl->mode;
    }
    return SEQCDC_OK;
  };
  // coordinate search: segment length, then mark span, then chain occupancy
  for (u64 m : {32ull, 64ull, 128ull, 256ull, 512ull, 1024ull})
    if ((rc = trial(m, 16, 16))) break;
  if (!rc) {
    const u64 m = best.seg_mult;
    for (u32 s : {8u, 32u, 64u})
      if ((rc = trial(m, s, 16))) break;
  }
  if (!rc) {
    const u64 m = best.seg_mult;
    const u32 s = best.span_blocks;
    for (u32 w : {8u, 12u, 20u})
      if ((rc = trial(m, s, w))) break;
  }
  if (!rc) {  // the direct (skip-aware) chains: no mark span; segment length and occupancy
    pl->mode = 1;
    const u64 m0 = best.seg_mult;
    const u32 s = best.span_blocks;
    for (u64 m : {m0 / 2, m0, m0 * 2})
      if (m >= 16 && (rc = trial(m, s, 12))) break;
    if (!rc) {
      const u64 m = best.mode == 1 ? best.seg_mult : m0;
      for (u32 w : {8u, 16u})
        if ((rc = trial(m, s, w))) break;
    }
  }
  if (!rc) {  // the fastest candidates again, each timed over more calls
    best.ms = 1e30;
    for (const Candidate& c : finalists(tried)) {
      pl->mode = c.mode;
      pl->seg_override = c.seg * p->min_size;
      pl->span_override = c.span;
      pl->waves_override = c.waves;
      double ms = 0;
      if ((rc = time_config(pl, d_sample, n, p, d_cuts, cap, st, e0, e1, kFinalReps, &ms))) break;
      if (ms < best.ms) {
        best.ms = ms;
        best.seg_mult = c.seg;
        best.span_blocks = c.span;
        best.waves_per_cu = c.waves;
        best.mode = c.mode;
      }
    }
  }
  pl->mode = saved_mode;
  pl->seg_override = saved_seg;
  pl->span_override = saved_span;
  pl->waves_override = saved_waves;
  if (!rc) {
    tune_store(best);
    if (best_ms) *best_ms = best.ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_cuts);
  return rc;
}

extern "C" int seqcdc_autotune_batch(seqcdc_plan* plan, const seqcdc_file* h_files, uint32_t nfiles,
                                     const seqcdc_params* h_params, uint32_t nparams, uint64_t* d_cuts,
                                     const uint64_t* h_cut_offsets, uint64_t* d_counts, double* best_ms,
                                     void* stream) {
  if (!plan) return fail(SEQCDC_EINVAL, "plan is NULL");
  if (!h_files || !h_params || !h_cut_offsets || nfiles == 0 || nparams == 0)
    return fail(SEQCDC_EINVAL, "empty batch");
  int rc;
  u64 min_min = ~0ull;
  for (u32 i = 0; i < nparams; i++) {
    if ((rc = validate(&h_params[i]))) return rc;
    min_min = std::min<u64>(min_min, h_params[i].min_size);
  }
  Plan* pl = (Plan*)plan;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const u64 saved_seg = pl->seg_override;
  const u32 saved_span = pl->span_override, saved_waves = pl->waves_override;
  const int saved_mode = pl->mode;
  double best = 1e30;
  u64 best_seg = 0;
  u32 best_span = 16, best_waves = 12;
  int best_mode = 0;
  std::vector<Candidate> tried;
  auto time_setting = [&](u64 seg, u32 span, u32 waves, int mode, int reps, double* ms) -> int {
    pl->seg_override = seg;
    pl->span_override = span;
    pl->waves_override = waves;
    pl->mode = mode;
    return time_batch(pl, h_files, nfiles, h_params, nparams, d_cuts, h_cut_offsets, d_counts, st, e0, e1, reps, ms);
  };
  auto trial = [&](u64 seg, u32 span, u32 waves, int mode) -> int {
    double ms = 0;
    int r = time_setting(seg, span, waves, mode, kTrialReps, &ms);
    if (r) return r;
    tried.push_back(Candidate{seg, span, waves, mode, ms});
    if (ms < best) {
      best = ms;
      best_seg = seg;
      best_span = span;
      best_waves = waves;
      best_mode = mode;
    }
    return SEQCDC_OK;
  };
  // coordinate search over the batch itself: segment length (multiples of
  // the smallest min_size), mark span, chain occupancy, then the direct mode
  rc = SEQCDC_OK;
  for (u64 m : {16ull, 32ull, 64ull, 128ull, 256ull})
    if ((rc = trial(m * min_min, 16, 12, 0))) break;
  if (!rc)
    for (u32 s : {8u, 32u})
      if ((rc = trial(best_seg, s, 12, 0))) break;
  if (!rc) {
    const u32 s = best_span;
    for (u32 w : {8u, 16u, 20u})
      if ((rc = trial(best_seg, s, w, 0))) break;
  }
  if (!rc) rc = trial(best_seg, best_span, 12, 1);
  if (!rc) {  // the fastest candidates again, each timed over more calls
    best = 1e30;
    for (const Candidate& c : finalists(tried)) {
      double ms = 0;
      if ((rc = time_setting(c.seg, c.span, c.waves, c.mode, kFinalReps, &ms))) break;
      if (ms < best) {
        best = ms;
        best_seg = c.seg;
        best_span = c.span;
        best_waves = c.waves;
        best_mode = c.mode;
      }
    }
  }
  if (!rc) {  // the plan keeps the fastest settings
    pl->seg_override = best_seg;
    pl->span_override = best_span;
    pl->waves_override = best_waves;
    pl->mode = best_mode;
    if (best_ms) *best_ms = best;
  } else {
    pl->seg_override = saved_seg;
    pl->span_override = saved_span;
    pl->waves_override = saved_waves;
    pl->mode = saved_mode;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
