// SeqCDC mark step on CDNA4 (gfx950): the stand-alone mark kernel, which
// writes the EO16 bitmaps of a stream without resolving cuts.  The chunking
// entry points mark inside the pipeline kernel instead, with the same device
// functions.

#include <hip/hip_runtime.h>

#include "seqcdc_mark.h"

namespace seqcdc {

// One wave per mark span; files are located by a binary search over their
// first span.
__global__ __launch_bounds__(256) void mark_kernel(const FileDesc* __restrict__ files, u32 nfiles, u64 total_spans,
                                                   u32 span_blocks) {
  const u64 span = (u64)blockIdx.x * kWavesPerGroup + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  if (span >= total_spans) return;
  const FileDesc& F = files[file_of_span(files, nfiles, span)];
  mark_span(F, span - F.mark_span0, span_blocks);
}

hipError_t launch_mark(const FileDesc* d_files, u32 nfiles, u64 total_spans, u32 span_blocks, hipStream_t st) {
  const u64 groups = (total_spans + kWavesPerGroup - 1) / kWavesPerGroup;
  hipLaunchKernelGGL(mark_kernel, dim3((u32)(groups ? groups : 1)), dim3(256), 0, st, d_files, nfiles, total_spans,
                     span_blocks);
  return hipGetLastError();
}

}  // namespace seqcdc
