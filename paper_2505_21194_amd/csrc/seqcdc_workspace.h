// Resolve-stage workspace shared by the HIP kernels and the host runtime of
// libseqcdc (not part of the public C ABI): per-chain state.
#pragma once
#include "seqcdc_internal.h"

namespace seqcdc {

// Per-chain workspace (indexed by global chain id).
struct ChainWs {
  u32* chain_file;     // file index of the chain
  u64* list;           // cut lists of multi-segment files
  u64* list_off;       // offset of each chain's list in `list`
  u32* list_cnt;       // entries in the chain's list (the last is its exit cut)
  u64* conv_val;       // boundary k: first cut of chain k's continuation found in a later chain
  u32* conv_chain;     // segment (relative) whose list holds conv_val; nseg = reached the end
  i32* conv_idx;       // index of conv_val in that list; -1 = the segment start itself
  u64* cont_cnt;       // continuation cuts before conv_val (more than cont_cap once the stitch took it further)
  u64* cont;           // continuation cuts, cont_cap per multi-segment chain
  u64* cont_off;       // offset of each chain's continuation buffer in `cont`
  u32 cont_cap;        // pass B stops a continuation whose buffer is full, leaving it open
  u64* ovf;            // overflow regions (FileDesc::ovf0): cuts of open continuations taken further by the stitch
  u64* ovf_start;      // where a chain's overflow cuts start in `ovf`
  u32* active;         // stitch: chain contributes to the output
  i32* entry_idx;      // stitch: index of the chain's first exact cut (-1 = segment start)
  u64* out_off;        // stitch: output offset of the chain's part
  u32* jumps;          // stitch scratch: (boundary, target chain) pairs of continuations that passed a whole segment
  u32* covered;        // stitch scratch: covered ranges (pairs)
};

}  // namespace seqcdc
