// Resolve-stage workspaces shared by the HIP kernels and the host runtime of
// libseqcdc (not part of the public C ABI): per-chain state and the ordered
// work list of the pipeline modes.
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
  u32* cont_cnt;       // continuation cuts before conv_val (may exceed cont_cap)
  u64* cont;           // continuation cuts, cont_cap per multi-segment chain
  u64* cont_off;       // offset of each chain's continuation buffer in `cont`
  u32 cont_cap;
  u32* active;         // stitch: chain contributes to the output
  i32* entry_idx;      // stitch: index of the chain's first exact cut (-1 = segment start)
  u64* out_off;        // stitch: output offset of the chain's part
  u32* jumps;          // stitch scratch: (boundary, target chain) pairs of continuations that passed a whole segment
  u32* covered;        // stitch scratch: covered ranges (pairs)
  const u32* stall;    // nonzero: a pass A could not finish (never expected); the results are void
};

// Work queue of the pipeline kernel.  Items are handed out in list order; an
// item is a mark span (its global index) or a chain (kItemChain | global
// chain id: pass A over its segment, then its continuation).  A wave waits
// only for items already handed out (their waves are running and never wait
// for later items), so the kernel cannot deadlock whatever the grid size.  A
// chain's item comes after every span its pass A can read; a continuation
// that reaches work not handed out yet stops and is resumed by a later kernel.
constexpr u32 kItemChain = 0x80000000u;

struct PipeWs {
  const u32* items;      // item codes in hand-out order
  u32 nitems;
  u32 span_blocks;       // 1 KiB mark blocks per span (a multiple of 4)
  const u32* span_pos;   // per global span: its position in `items`
  const u32* chain_pos;  // per global chain: its position in `items`
  u32* head;             // next list position to hand out
  u32* span_done;        // per global span: bits written and released
  u32* chain_done;       // per global chain: pass A list published
  u32* resume;           // resume list and counters, indexed by the constants below
  u32 premarked;         // every span was marked by an earlier kernel: the list holds chains only
  u32 wait_rounds;       // bound of every wait on a flag (rounds of a short sleep)
};

constexpr u32 kResumeCount = 0;  // continuations to resume
constexpr u32 kResumeHead = 1;   // resume kernel's hand-out head
constexpr u32 kStall = 2;        // a pass A could not finish
constexpr u32 kTimeouts = 3;     // bounded waits that ran out
constexpr u32 kResumeList = 16;  // chain ids to resume

}  // namespace seqcdc
