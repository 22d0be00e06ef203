// Internal descriptors shared by the HIP kernels and the host runtime of
// libseqcdc (not part of the public C ABI).
#pragma once
#include <stdint.h>

namespace seqcdc {

typedef uint32_t u32;
typedef uint64_t u64;
typedef int32_t i32;

constexpr u32 kNoSkip = 0xFFFFFFFFu;
constexpr u32 kWaveSize = 64;
constexpr u32 kMarkBlock = 1024;  // bytes per wave per mark step (64 lanes x 16 B)
constexpr u32 kWavesPerGroup = 4;  // 256-thread workgroups
constexpr u32 kHintSpans = 64;     // mark spans per entry of the span -> file hint table

// One stream ("file") of a batch, as the kernels see it.
//
// Mark bitmap layout ("EO16"): byte q of the file belongs to group q/64; a
// group is 4 dwords and dword j holds E bits (low half) and O bits (high
// half) of the 16 bytes 64g+16j .. 64g+16j+15, bit i <-> byte 64g+16j+i.
struct FileDesc {
  const uint8_t* data;  // caller's bytes
  u64 n;                // length in bytes
  u32* eo;              // 4 * ceil(n/64) dwords of mark bits
  uint8_t* esum;        // ceil(n/1024) bytes (+ padding to 16): block holds a run end
  u32 mode;             // 0 increasing, 1 decreasing
  u32 sl;               // SeqLength (bytes in the run), 2..16
  u64 min_size, max_size;
  u32 trig;             // SkipTrigger, kNoSkip = off
  u32 skip;             // SkipSize
  u64 mark_span0;       // global index of the file's first mark span
  u64 seg;              // segment length for speculative chains
  u32 nseg;             // number of segments (chains)
  u32 chain0;           // global index of chain 0 of this file
  u64* out;             // final cut list destination
  u64 out_cap;          // entries available at out
  u64* out_count;       // where the final count is written (device)
};

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
  u32* jumps;          // stitch scratch: boundaries whose continuation passed a whole segment
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
