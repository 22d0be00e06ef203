// Monte-Carlo calibration of SeqCDC's parameters (Sec. V, Table I): the
// paper picks SeqLength, SkipTrigger and SkipSize so that random data gives
// the target average chunk size.  Here one device-resident sample is chunked
// under every candidate parameter set in one batched call (each candidate is
// a "file" of the batch over the same bytes), and a reduction kernel gathers
// each candidate's chunk statistics on the device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_device.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

// Per candidate: chunks, chunks cut at max_size (not counting the last chunk),
// sum of squared chunk lengths.
struct CalibAcc {
  unsigned long long chunks, at_max, sumsq;
  unsigned long long pad;
};

// One thread per cut slot of candidate c = blockIdx.y: the chunk ending at
// that cut, reduced over the wave before one atomic per wave and quantity.
__global__ __launch_bounds__(256) void calib_stats_kernel(const u64* __restrict__ cuts, const u64* __restrict__ offs,
                                                          const u64* __restrict__ counts,
                                                          const u64* __restrict__ max_size, CalibAcc* acc) {
  const u32 c = blockIdx.y;
  const u64 j = (u64)blockIdx.x * 256 + threadIdx.x;
  const u64 cnt = counts[c];
  u64 len = 0;
  bool valid = j < cnt;
  if (valid) {
    const u64* cc = cuts + offs[c];
    len = cc[j] - (j ? cc[j - 1] : 0);
  }
  const bool at_max = valid && j + 1 < cnt && len == max_size[c];
  // wave sums: chunks and maximum-size chunks by ballot, squares by a DPP scan of the halves
  const u64 n_valid = __popcll(ballot(valid));
  const u64 n_max = __popcll(ballot(at_max));
  const u64 sq = len * len;  // < 2^61 for chunks below 1 GiB
  const u64 tot = wave_incl_scan64(sq);
  if (lane_id() == 63) {
    if (n_valid) atomicAdd(&acc[c].chunks, (unsigned long long)n_valid);
    if (n_max) atomicAdd(&acc[c].at_max, (unsigned long long)n_max);
    if (tot) atomicAdd(&acc[c].sumsq, (unsigned long long)tot);
  }
}

__global__ void calib_clear_kernel(CalibAcc* acc, u32 n) {
  for (u32 i = threadIdx.x; i < n; i += blockDim.x) acc[i] = CalibAcc{0, 0, 0, 0};
}

}  // namespace seqcdc

using namespace seqcdc;

extern "C" int seqcdc_calibrate(seqcdc_plan* plan, const void* d_sample, uint64_t n, const seqcdc_params* cands,
                                uint32_t ncand, seqcdc_calib_stats* out, void* stream) {
  if (!plan || !cands || !out) return fail(SEQCDC_EINVAL, "NULL argument");
  if (!d_sample || n == 0) return fail(SEQCDC_EINVAL, "empty sample");
  if (ncand == 0) return SEQCDC_OK;
  if (ncand > 65535) return fail(SEQCDC_EINVAL, "at most 65535 candidates");
  int rc;
  for (u32 i = 0; i < ncand; i++)
    if ((rc = validate(&cands[i]))) return rc;
  Plan* pl = (Plan*)plan;
  hipStream_t st = (hipStream_t)stream;
  // cut ranges of the candidates, laid out one after the other
  std::vector<u64> offs(ncand + 1, 0), maxs(ncand);
  u64 most = 0;
  for (u32 i = 0; i < ncand; i++) {
    const u64 m = max_cuts(n, &cands[i]);
    offs[i + 1] = offs[i] + m;
    maxs[i] = cands[i].max_size;
    most = std::max<u64>(most, m);
  }
  std::vector<seqcdc_file> files(ncand);
  for (u32 i = 0; i < ncand; i++) files[i] = seqcdc_file{d_sample, n, i, 0};
  const size_t cut_bytes = offs[ncand] * 8;
  const size_t tab = (3 * ncand + 1) * 8;
  {
    std::lock_guard<std::mutex> g(pl->mu);
    if ((rc = pl->aux.reserve(cut_bytes + 256 + tab + 256 + ncand * sizeof(CalibAcc)))) return rc;
    if ((rc = pl->aux_host.reserve(tab + ncand * sizeof(CalibAcc)))) return rc;
  }
  char* base = (char*)pl->aux.p;
  u64* d_cuts = (u64*)base;
  u64* d_tab = (u64*)(base + ((cut_bytes + 255) & ~(size_t)255));
  u64* d_counts = d_tab;                // ncand
  u64* d_offs = d_tab + ncand;          // ncand + 1
  u64* d_max = d_tab + 2 * ncand + 1;   // ncand
  CalibAcc* d_acc = (CalibAcc*)((char*)d_tab + ((tab + 255) & ~(size_t)255));
  // one batched chunking call over all candidates (it orders this stream after the plan's earlier calls)
  if ((rc = chunk_batch(pl, files.data(), ncand, cands, ncand, d_cuts, offs.data(), d_counts, st))) return rc;
  std::lock_guard<std::mutex> g(pl->mu);
  u64* h = (u64*)pl->aux_host.p;
  for (u32 i = 0; i <= ncand; i++) h[ncand + i] = offs[i];
  for (u32 i = 0; i < ncand; i++) h[2 * ncand + 1 + i] = maxs[i];
  hipError_t e = hipMemcpyAsync(d_offs, h + ncand, (2 * ncand + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(calib_clear_kernel, dim3(1), dim3(256), 0, st, d_acc, ncand);
    hipLaunchKernelGGL(calib_stats_kernel, dim3((u32)((most + 255) / 256), ncand), dim3(256), 0, st, d_cuts, d_offs,
                       d_counts, d_max, d_acc);
    e = hipGetLastError();
  }
  CalibAcc* hacc = (CalibAcc*)(h + 3 * ncand + 1);
  if (e == hipSuccess) e = hipMemcpyAsync(hacc, d_acc, ncand * sizeof(CalibAcc), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "seqcdc_calibrate");
  pl->pending = false;
  pl->upload_pending = false;
  for (u32 i = 0; i < ncand; i++) {
    const double k = (double)hacc[i].chunks;
    out[i].chunks = hacc[i].chunks;
    out[i].max_chunks = hacc[i].at_max;
    out[i].mean = k > 0 ? (double)n / k : 0.0;
    const double var = k > 0 ? (double)hacc[i].sumsq / k - out[i].mean * out[i].mean : 0.0;
    out[i].stddev = var > 0 ? sqrt(var) : 0.0;
  }
  return SEQCDC_OK;
}
