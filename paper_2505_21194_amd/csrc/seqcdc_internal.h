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
  u32 mode;             // bit 0: decreasing; bit 1: bytes compared as signed values
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
  u64 ovf0;             // multi-segment files: first entry of the file's overflow region (n/min_size + 2 entries)
};

}  // namespace seqcdc
