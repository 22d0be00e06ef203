// Host-side launchers of the mark and resolve kernels (defined next to the
// kernels); every pointer is a device pointer.
#pragma once
#include <hip/hip_runtime.h>

#include "seqcdc_internal.h"
#include "seqcdc_workspace.h"

namespace seqcdc {

hipError_t launch_mark(const FileDesc* d_files, const u32* d_hint, u64 span_lo, u64 span_hi, u32 span_blocks,
                       hipStream_t st);
hipError_t launch_clear(u32* p, u64 count, hipStream_t st);
// direct: the skip-aware chains that read raw input windows (no mark pass);
// otherwise the chains read the mark kernel's bits.
hipError_t launch_chains(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32* head,
                         u32 groups, bool direct, hipStream_t st);
hipError_t launch_continue(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32* head,
                           u32 groups, bool direct, hipStream_t st);
hipError_t launch_stitch(const FileDesc* d_files, const ChainWs& ws, const u32* d_multi, u32 nmulti, bool direct,
                         hipStream_t st);
hipError_t launch_compact(const FileDesc* d_files, const ChainWs& ws, const u32* d_chains, u32 nchains,
                          hipStream_t st);

}  // namespace seqcdc
