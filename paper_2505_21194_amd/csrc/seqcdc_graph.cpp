// Prepared batches: a batch whose files, parameters and output arrays stay
// the same from launch to launch (a ring of device buffers refilled with new
// data, a fixed set of volumes) is laid out once, in a workspace of its own,
// and its launch sequence (counter clearing, mark, pass A, pass B, stitch,
// compaction) is captured into a hipGraph.  A launch replays the graph: no
// host-side layout, no table upload, one submission.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "seqcdc_runtime.h"

namespace seqcdc {

struct Batch {
  Plan plan;  // private: owns the workspace the graph's kernels point into
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // after the last launch
  bool launched = false;
  std::mutex mu;
};

static void batch_free(Batch* b) {
  if (b->launched) (void)hipEventSynchronize(b->done);
  if (b->cap) (void)hipStreamSynchronize(b->cap);  // a preparation that failed half-way may have work in flight
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->done) (void)hipEventDestroy(b->done);
  plan_free(&b->plan);
  delete b;
}

static int prepare(Plan* settings, const seqcdc_file* files, u32 nfiles, const seqcdc_params* params, u32 nparams,
                   u64* d_cuts, const u64* h_off, u64* d_counts, Batch** out) {
  std::vector<Spec> specs;
  int rc;
  if ((rc = build_specs(files, nfiles, params, nparams, d_cuts, h_off, d_counts, specs))) return rc;
  int dev = -1;
  if (settings) {
    std::lock_guard<std::mutex> g(settings->mu);
    dev = settings->device;
  }
  Batch* b = new Batch();
  if ((rc = plan_init(&b->plan, dev))) {
    delete b;
    return rc;
  }
  Plan& pl = b->plan;
  if (settings) {  // the caller's tuning choices and resolve mode as that plan would pick them
    std::lock_guard<std::mutex> g(settings->mu);
    pl.seg_override = settings->seg_override;
    pl.span_override = settings->span_override;
    pl.waves_override = settings->waves_override;
    pl.mode = settings->mode_for(params);
  }
  pl.overlap = 1;  // one stream: the graph is a single chain of kernels
  auto hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) rc = hip_fail(e, what);
    return e == hipSuccess;
  };
  if (!hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "hipStreamCreateWithFlags") ||
      !hip(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "hipEventCreateWithFlags")) {
    batch_free(b);
    return rc;
  }
  // An eager call sizes and fills the workspace (and runs the batch once).
  if ((rc = run_batch(&pl, specs.data(), nfiles, b->cap, false)) ||
      !hip(hipStreamSynchronize(b->cap), "hipStreamSynchronize")) {
    batch_free(b);
    return rc;
  }
  pl.pending = false;
  pl.upload_pending = false;
  // The same call again under stream capture: the layout is identical, so no
  // buffer grows and the tables already on the device are the ones it uses.
  if (!hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")) {
    batch_free(b);
    return rc;
  }
  pl.capturing = true;
  const int run_rc = run_batch(&pl, specs.data(), nfiles, b->cap, false);
  pl.capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t end = hipStreamEndCapture(b->cap, &graph);
  b->graph = graph;
  if (run_rc) {
    batch_free(b);
    return run_rc;
  }
  if (!hip(end, "hipStreamEndCapture") ||
      !hip(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate")) {
    batch_free(b);
    return rc;
  }
  *out = b;
  return SEQCDC_OK;
}

}  // namespace seqcdc

using namespace seqcdc;

extern "C" {

int seqcdc_batch_prepare(seqcdc_plan* settings, const seqcdc_file* files, uint32_t nfiles,
                         const seqcdc_params* params, uint32_t nparams, uint64_t* d_cuts,
                         const uint64_t* h_cut_offsets, uint64_t* d_counts, seqcdc_batch** out) {
  if (!out) return fail(SEQCDC_EINVAL, "out is NULL");
  *out = nullptr;
  if (nfiles == 0) return fail(SEQCDC_EINVAL, "a prepared batch needs at least one file");
  Batch* b = nullptr;
  const int rc = prepare((Plan*)settings, files, nfiles, params, nparams, d_cuts, h_cut_offsets, d_counts, &b);
  if (rc) return rc;
  *out = (seqcdc_batch*)b;
  return SEQCDC_OK;
}

int seqcdc_batch_launch(seqcdc_batch* batch, void* stream) {
  if (!batch) return fail(SEQCDC_EINVAL, "batch is NULL");
  Batch* b = (Batch*)batch;
  std::lock_guard<std::mutex> g(b->mu);
  hipError_t e = hipSetDevice(b->plan.device);
  // launches share the batch's workspace: each one starts after the previous one, whatever its stream
  if (e == hipSuccess && b->launched) e = hipStreamWaitEvent((hipStream_t)stream, b->done, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e == hipSuccess) e = hipEventRecord(b->done, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  b->launched = true;
  return SEQCDC_OK;
}

int seqcdc_batch_destroy(seqcdc_batch* batch) {
  if (!batch) return fail(SEQCDC_EINVAL, "batch is NULL");
  batch_free((Batch*)batch);
  return SEQCDC_OK;
}

}  // extern "C"
