// SeqCDC mark step on CDNA4 (gfx950): the mark kernel, which writes the EO16
// bitmaps and run-end summary of every file of a call.

#include <hip/hip_runtime.h>

#include "seqcdc_mark.h"

namespace seqcdc {

// One wave per mark span of [span_lo, span_hi) (global span indices); files
// are located through the span hint table.
__global__ __launch_bounds__(256) void mark_kernel(const FileDesc* __restrict__ files, const u32* __restrict__ hint,
                                                   u64 span_lo, u64 span_hi, u32 span_blocks) {
  const u64 span = span_lo + (u64)blockIdx.x * kWavesPerGroup +
                   __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  if (span >= span_hi) return;
  const FileDesc& F = files[file_of_span(files, hint, span)];
  mark_span(F, span - F.mark_span0, span_blocks);
}

hipError_t launch_mark(const FileDesc* d_files, const u32* d_hint, u64 span_lo, u64 span_hi, u32 span_blocks,
                       hipStream_t st) {
  if (span_hi <= span_lo) return hipSuccess;
  const u64 groups = (span_hi - span_lo + kWavesPerGroup - 1) / kWavesPerGroup;
  hipLaunchKernelGGL(mark_kernel, dim3((u32)groups), dim3(256), 0, st, d_files, d_hint, span_lo, span_hi,
                     span_blocks);
  return hipGetLastError();
}

}  // namespace seqcdc
