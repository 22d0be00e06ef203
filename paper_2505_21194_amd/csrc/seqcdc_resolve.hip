// SeqCDC resolve step on CDNA4 (gfx950): the exact sequential state machine
// of the paper run over the mark bits, speculatively per segment.
//
// From a cut at c (Sec. III-B) scanning starts at s = c + min - SeqLength;
// the chunk ends one byte past the first run end E at or after s+SeqLength-1
// (Sec. III-A), unless the SkipTrigger-th opposing pair O after s comes first,
// in which case SkipSize bytes after it are not scanned and scanning restarts
// with fresh counters (Sec. III-C); nothing is scanned at or past
// min(c + max, n) (Sec. IV).  Only the first event in byte order matters: a
// pair cannot be favourable and opposing at once.
//
// Parallelism: a stream is split into segments.  A chain starts at every
// segment start as if a cut were there (pass A).  The state after a cut
// depends only on the cut's position, so once two chains share a cut they
// agree from then on.  Pass B continues each chain past its segment until one
// of its cuts belongs to the chain that owns that position; the stitch then
// keeps the exact pieces and the compaction writes them out.  Every
// dependency between workgroups is a kernel boundary: mark, pass A, pass B,
// stitch and compaction are separate launches, and the only shared state
// inside a launch is its atomic work counter.
//
// A chain is one wave, and the waves of a workgroup take chains
// independently.  Its state is wave-uniform (scalar registers); the lanes
// hold one window of run-end and opposing bits, one group of bytes per lane,
// with per-window prefix counts, so every scan step is a handful of lane reads
// and scalar operations.  Two kinds of window feed the same state machine:
//  - marked (MarkedChain): 4 KiB of bits the mark kernel wrote (EO16), one
//    64-byte group per lane.  A per-1 KiB summary of run ends lets a chain
//    cross regions with no run end (zero runs, most short periodic patterns)
//    without reading their bits: with no run end before the limit, the chunk
//    ends at the limit whatever the opposing pairs do.
//  - direct (DirectChain, skip-aware): 1 KiB of raw input bytes, one 16-byte
//    group per lane, whose bits the chain computes itself when it enters the
//    window.  There is no mark pass: only the windows a chain scans are read
//    from HBM, so the sub-minimum region after each cut and the bytes a skip
//    passes over are never loaded (Sec. III-B, III-C).

#include <hip/hip_runtime.h>

#include "seqcdc_mark.h"
#include "seqcdc_workspace.h"

namespace seqcdc {

constexpr u32 kSubBytes = 4096;  // input bytes per sub-window: 64 groups, one per lane
constexpr u32 kRing = 8;         // LDS slots per wave: sub-window w lives in slot w % kRing

__device__ __forceinline__ u64 min64(u64 a, u64 b) { return a < b ? a : b; }

// A wave-uniform 32-bit value the optimiser may not look through (an empty
// asm statement, no instruction): compares built from the 32-bit halves of a
// 64-bit value stay scalar compares.  The scalar unit has no ordered 64-bit
// compare, and recombined into one they would run on the vector unit.
__device__ __forceinline__ u32 opaque_u32(u32 v) {
  asm("" : "+s"(v));
  return v;
}

// a < b for 64-bit positions less than 2^63 apart, on the scalar unit.
__device__ __forceinline__ bool before(u64 a, u64 b) { return opaque_u32((u32)((a - b) >> 32)) >= 0x80000000u; }
__device__ __forceinline__ u64 max64(u64 a, u64 b) { return a > b ? a : b; }

// Position of the k-th (1-based) set bit of a wave-uniform word w: lane b
// counts the set bits of w below b (mbcnt); the lanes with fewer than k such
// bits are exactly 0 .. position.
__device__ __forceinline__ u32 select_bit(u64 w, u32 k) {
  const u32 below = __builtin_amdgcn_mbcnt_hi((u32)(w >> 32), __builtin_amdgcn_mbcnt_lo((u32)w, 0u));
  return (u32)__popcll(ballot(below < k)) - 1;
}

// E (run ends) and O (opposing pairs) of one group from its EO16 dwords.
__device__ __forceinline__ void unpack_group(const uint4& v, u64& E, u64& O) {
  E = (u64)__builtin_amdgcn_perm(v.y, v.x, 0x05040100u) | ((u64)__builtin_amdgcn_perm(v.w, v.z, 0x05040100u) << 32);
  O = (u64)__builtin_amdgcn_perm(v.y, v.x, 0x07060302u) | ((u64)__builtin_amdgcn_perm(v.w, v.z, 0x07060302u) << 32);
}

// ---------------------------------------------------------------------------
// The chain
// ---------------------------------------------------------------------------

// Wave-uniform state (scalar registers) plus one sub-window of bits in the
// lanes.  Indices of 64-byte groups, 1 KiB blocks and 4 KiB sub-windows are
// 32-bit (streams are shorter than 256 GiB) and chunk-relative offsets are
// 32-bit (max_size <= 1 GiB), so the state fits the scalar register file.
struct MarkedChain {
  static constexpr u32 kWin = kSubBytes;  // bytes per window
  static constexpr u32 kG = 64;           // bytes per lane group
  static constexpr bool kSummary = true;  // has the run-end summary
  typedef u64 Word;                       // E / O bits of one group
  const uint4* eo;    // EO16 groups of the file
  const uint8_t* esum;
  u64 n;
  u32 groups;
  u32 min_size, max_size, sl, trig, skip;
  u32 cur;            // sub-window held in E/O (kNone = none)
  u32 pf_base;        // bit i of pf_mask: the DMA of sub-window pf_base + i into its slot was issued
  u32 pf_mask;
  SEQCDC_LOCAL u32x4* win;  // this wave's kRing LDS window slots (kRing x 64 groups)
  u64 E, O;           // lane l: group cur*64 + l
  u32 incl;           // lane l: opposing pairs in groups 0..l of the window (inclusive prefix)
  u32 excl;           // lane l: opposing pairs in groups 0..l-1 of the window
  u32 fe;             // lane l: first run-end bit of the group (64 = none)
  u32 total;          // opposing pairs in the whole window
  u64 emask;          // bit l: group l holds a run end
  // summary knowledge, 0 = none, else (to << 1) | hit: the blocks from the
  // last one asked about up to `to` hold no run end, and hit says whether
  // `to` is a block with a run end (or the end) rather than a horizon.  A
  // chain asks about blocks in increasing order, so the knowledge holds for
  // every later question up to `to`.
  u32 sumk;
};

constexpr u32 kNone = 0xFFFFFFFFu;

template <class Ch>
__device__ __forceinline__ bool skipping(const Ch& ch) { return ch.trig != kNoSkip; }

__device__ __forceinline__ void chain_init(MarkedChain& ch, const FileDesc& F, SEQCDC_LOCAL u32x4* win) {
  ch.win = win;
  ch.eo = (const uint4*)F.eo;
  ch.esum = F.esum;
  ch.n = F.n;
  ch.groups = (u32)((F.n + 63) >> 6);
  ch.min_size = (u32)F.min_size;
  ch.max_size = (u32)F.max_size;
  ch.sl = F.sl;
  ch.trig = F.trig;
  ch.skip = F.skip;
  ch.cur = kNone;
  ch.pf_base = 0;
  ch.pf_mask = 0;
  ch.E = ch.O = 0;
  ch.incl = ch.excl = ch.total = 0;
  ch.fe = 64;
  ch.emask = 0;
  ch.sumk = 0;
}

// Starts the DMA of sub-window `sub` into its LDS slot (sub % kRing): lane l
// copies group sub*64 + l.  Lanes past the end read the last group instead
// (always in bounds); their data is discarded when the slot is read.
__device__ __forceinline__ void dma_window(const MarkedChain& ch, u32 sub) {
  const u32 g = sub * 64u + lane_id();
  const u32 gs = g < ch.groups ? g : ch.groups - 1;
  __builtin_amdgcn_global_load_lds(as_global((const void*)(ch.eo + gs)), ch.win + (sub & (kRing - 1)) * 64, 16, 0,
                                   0);
}

// Loads sub-window `sub` and its per-window facts.  On entry to a window the
// DMAs of the windows the chain is likely to need next are started: the next
// one (the scan continues) and the two from `hint` on, the sub-window where
// the scan would restart if a cut were found right at the current position (a
// cut is usually a few hundred bytes away, and the scan after it starts
// min_size - SeqLength bytes later).  Windows are entered in increasing
// order, so the slots of the kRing - 1 windows after `sub` never collide.
__device__ __forceinline__ void ensure(MarkedChain& ch, u32 sub, u32 hint) {
  if (ch.cur == sub) return;
  const u32 d = sub - ch.pf_base;
  u32 mask = d < kRing ? ch.pf_mask >> d : 0u;
  if (!(mask & 1u)) dma_window(ch, sub);
  SEQCDC_WAIT_VMEM();
  const u32x4 w = ch.win[(sub & (kRing - 1)) * 64 + lane_id()];
  const bool inside = sub * 64u + lane_id() < ch.groups;
  const uint4 v = inside ? make_uint4(w.x, w.y, w.z, w.w) : make_uint4(0, 0, 0, 0);
  mask |= 1u;  // sub itself sits in its slot now
  // windows worth fetching ahead: sub+1, hint and hint+1, inside the stream
  u32 want = 2u;
  const u32 hi = hint - sub;  // hint >= sub
  if (hi < kRing - 1) want |= 3u << hi;
  const u32 nwin = (ch.groups + 63) >> 6;
  const u32 room = nwin > sub ? nwin - sub : 0u;
  if (room < kRing) want &= (1u << room) - 1u;
  want &= ~mask;
  mask |= want;
  while (want) {
    dma_window(ch, sub + (u32)__builtin_ctz(want));
    want &= want - 1u;
  }
  ch.pf_base = sub;
  ch.pf_mask = mask;
  unpack_group(v, ch.E, ch.O);
  ch.cur = sub;
  // per-window facts every scan of this window reuses
  ch.emask = ballot(ch.E != 0);
  ch.fe = ch.E ? ctz64(ch.E) : 64u;
  if (skipping(ch)) {
    const u32 cnt = (u32)__popcll(ch.O);
    ch.incl = wave_incl_scan(cnt);
    ch.excl = ch.incl - cnt;
    ch.total = readlane(ch.incl, 63);
  }
}

// One load of the summary from block b (up to 1024 blocks, 1 MiB of input):
// `to` becomes the first block at or after b holding a run end (hit), or the
// horizon of the load (blocks [b, to) hold no run end).
__device__ __forceinline__ void summary_load(const uint8_t* esum, u32 nb, u32 b, u32& to, bool& hit) {
  const u32 lane = lane_id();
  to = b;
  hit = b >= nb;
  if (b < nb) {
    const u32 a = b & ~15u;
    const u32 idx = a + 16u * lane;
    // branch-free (keeps the chain state wave-uniform): every lane reads a valid
    // 16-byte chunk of the padded summary; bytes outside [b, nb) are masked
    const uint4 v = load16(esum + (idx < nb ? idx : ((nb - 1) & ~15u)));
    const u32 d[4] = {v.x, v.y, v.z, v.w};
    u32 m = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const u32 t = d[k] & 0x01010101u;
      m |= ((t | (t >> 7) | (t >> 14) | (t >> 21)) & 0xFu) << (4 * k);
    }
    const u32 lo_sh = idx < b ? b - idx : 0u;  // < 16, only in lane 0
    m &= 0xFFFFu << lo_sh;
    const u32 room = idx < nb ? nb - idx : 0u;
    m = room < 16 ? (m & ((1u << room) - 1u)) : m;
    const u64 bal = ballot(m != 0);
    if (bal) {
      const u32 l = ctz64(bal);
      to = a + 16u * l + (u32)__builtin_ctz(readlane(m, l));
      hit = true;
    } else {
      to = a + 1024 < nb ? a + 1024 : nb;
      hit = to >= nb;
    }
  }
}

// True if no block in [b, ceil(L/1024)) holds a run end.  Uses and extends
// the summary knowledge; cheap when it already covers b.  Block indices are
// compared in 32 bits: to * 1024 >= L exactly when to >= ceil(L / 1024).
__device__ __forceinline__ bool no_end_before(MarkedChain& ch, u32 b, u64 L) {
  const u32 lb = (u32)((L + 1023) >> 10);
  u32 to = ch.sumk >> 1;
  bool hit = ch.sumk & 1u;
  u32 from = to;
  if (!ch.sumk || b > to) {
    from = b;
    hit = false;
    to = 0;
  }
  while (!hit && to < lb) {  // the first pass loads from b when the knowledge does not cover it
    summary_load(ch.esum, (u32)((ch.n + 1023) >> 10), from, to, hit);
    from = to;
  }
  ch.sumk = (to << 1) | (hit ? 1u : 0u);
  return to >= lb;
}

// ---------------------------------------------------------------------------
// The direct (skip-aware) chain: raw 1 KiB windows, bits computed on entry
// ---------------------------------------------------------------------------

constexpr u32 kDirectWin = 1024;                 // input bytes per window: 64 lanes x 16
constexpr u32 kDirectSlots = 8;                  // LDS window slots per wave
constexpr u32 kDirectSlotChunks = 66;            // aligned 16-byte chunks per slot
constexpr u32 kDirectLdsChunks = kDirectSlots * kDirectSlotChunks;

// Slots hold the aligned 16-byte chunks 64w - 1 .. 64w + 64 of window w
// (counted from the aligned address at or below the file's first byte): the
// window's 1 KiB wherever it starts within a chunk, plus the 16 bytes before
// it (the predecessors of lane 0's bytes).  Any slot holds any window; lane
// i < kDirectSlots of `tag` names the window in slot i.  Windows are entered
// in increasing order, so a slot holding a window below the current one is
// free.  No fetch is ever issued into a slot whose earlier fetch may still be
// in flight: prefetches are issued right after a wait for all earlier ones,
// into slots that were free then; a window that was not prefetched goes into
// the current window's slot, whose fetch completed before it was read; and a
// new chain first waits for the fetches its wave left in flight.
struct DirectChain {
  static constexpr u32 kWin = kDirectWin;
  static constexpr u32 kG = 16;
  static constexpr bool kSummary = false;
  typedef u32 Word;
  const uint8_t* base;  // aligned address at or below the file's first byte
  u64 last_chunk;       // chunks 0 .. last_chunk overlap the file (n > 0)
  u64 n;
  u32 nwin;             // ceil(n / 1024)
  u32 r;                // first byte's offset in its chunk (0..15)
  u32 down_is_fav;      // decreasing mode
  u32 flip;             // 0x80808080 for signed bytes (x ^ 0x80 orders as the signed value), else 0
  u32 min_size, max_size, sl, trig, skip;
  u32 cur;              // window whose bits are held (kNone = none)
  u32 cur_slot;         // its slot
  u32 tag;              // lane i < kDirectSlots: window held by slot i (kNone = empty)
  SEQCDC_LOCAL u32x4* win;  // kDirectSlots slots of kDirectSlotChunks chunks
  u32 E, O;             // lane l: bits of bytes 16l .. 16l+15 of the window (16 each)
  u32 incl, excl, fe, total;
  u64 emask;
};

__device__ __forceinline__ void chain_init(DirectChain& ch, const FileDesc& F, SEQCDC_LOCAL u32x4* win) {
  const uintptr_t addr = (uintptr_t)F.data;
  ch.r = (u32)(addr & 15);
  ch.base = (const uint8_t*)(addr - ch.r);
  ch.n = F.n;
  ch.last_chunk = F.n ? (ch.r + F.n - 1) >> 4 : 0;
  ch.nwin = (u32)((F.n + kDirectWin - 1) / kDirectWin);
  ch.down_is_fav = F.mode & 1;
  ch.flip = (F.mode & 2) ? 0x80808080u : 0u;
  ch.min_size = (u32)F.min_size;
  ch.max_size = (u32)F.max_size;
  ch.sl = F.sl;
  ch.trig = F.trig;
  ch.skip = F.skip;
  ch.cur = kNone;
  ch.cur_slot = 0;
  ch.tag = kNone;
  ch.win = win;
  SEQCDC_WAIT_VMEM();  // fetches of the wave's previous chain
  ch.E = ch.O = 0;
  ch.incl = ch.excl = ch.total = 0;
  ch.fe = 16;
  ch.emask = 0;
}

// Starts the DMA of window w into slot s: lane l copies chunk 64w - 1 + l into
// slot chunk l, lanes 0 and 1 chunks 64w + 63 and 64w + 64 into slot chunks 64
// and 65.  Chunks outside the file are clamped to its first or last chunk
// (always in bounds: a 16-byte aligned chunk never straddles a page); bytes
// outside the file are masked when the bits are computed.
__device__ __forceinline__ void dma_raw(const DirectChain& ch, u32 w, u32 s) {
  const u32 lane = lane_id();
  SEQCDC_LOCAL u32x4* dst = ch.win + s * kDirectSlotChunks;
  const u64 first = (u64)w * 64;  // chunk index of the window's slot chunk 1
  const u64 g = first + lane;     // slot chunk `lane` is chunk g - 1
  const u64 gm = g == 0 ? 0 : (g - 1 < ch.last_chunk ? g - 1 : ch.last_chunk);
  __builtin_amdgcn_global_load_lds(as_global((const void*)(ch.base + 16 * gm)), dst, 16, 0, 0);
  if (lane < 2) {
    const u64 t = first + 63 + lane;
    const u64 tm = t < ch.last_chunk ? t : ch.last_chunk;
    __builtin_amdgcn_global_load_lds(as_global((const void*)(ch.base + 16 * tm)), dst + 64, 16, 0, 0);
  }
}

// Slot holding window w, or kNone.
__device__ __forceinline__ u32 slot_of(const DirectChain& ch, u32 w) {
  const u64 m = ballot(lane_id() < kDirectSlots && ch.tag == w);
  return m ? ctz64(m) : kNone;
}

// Starts fetching window w into a free slot if it is in the file, not held
// and a slot is free (never the slot of window `keep`).
__device__ __forceinline__ void prefetch_raw(DirectChain& ch, u32 w, u32 keep) {
  if (w >= ch.nwin) return;
  const u32 lane = lane_id();
  const u64 held = ballot(lane < kDirectSlots && ch.tag == w);
  const u64 free = ballot(lane < kDirectSlots && (ch.tag == kNone || ch.tag < keep));
  if (held || !free) return;
  const u32 s = ctz64(free);
  dma_raw(ch, w, s);
  if (lane == s) ch.tag = w;
}

// Loads window w and computes its bits and per-window facts.  On entry the
// fetches of the windows the chain is likely to need next are started: the
// next one (the scan continues) and the two from `hint` on, the window where
// the scan would restart if a cut were found right at the current position (a
// cut is usually a few hundred bytes away, and the scan after it starts
// min_size - SeqLength bytes later).
__device__ __forceinline__ void ensure(DirectChain& ch, u32 w, u32 hint) {
  if (ch.cur == w) return;
  const u32 lane = lane_id();
  u32 s = slot_of(ch, w);
  if (s == kNone) {  // not prefetched: into the slot of the window entered before (slot 0 in a new chain)
    s = ch.cur_slot;
    dma_raw(ch, w, s);
    if (lane == s) ch.tag = w;
  }
  ch.cur_slot = s;
  SEQCDC_WAIT_VMEM();
  // lane l's 16 bytes and the 16 before them: slot bytes r + 16l .. r + 16l + 31,
  // read as 9 aligned dwords and realigned
  const SEQCDC_LOCAL u32* sw = (const SEQCDC_LOCAL u32*)(ch.win + s * kDirectSlotChunks);
  const u32 d0 = (ch.r + 16 * lane) >> 2, sh = ch.r & 3;
  u32 dw[9];
#pragma unroll
  for (int k = 0; k < 9; k++) dw[k] = sw[d0 + k];
  u32 halo[4], x[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    halo[k] = __builtin_amdgcn_alignbyte(dw[k + 1], dw[k], sh) ^ ch.flip;
    x[k] = __builtin_amdgcn_alignbyte(dw[k + 5], dw[k + 4], sh) ^ ch.flip;
  }
  // the next fetches go to other slots while the bits are computed
  prefetch_raw(ch, w + 1, w);
  prefetch_raw(ch, hint, w);
  prefetch_raw(ch, hint + 1, w);
  // Sec. III-D: favourable / opposing pairs, then run ends of SeqLength bytes
  u32 up, dn, hup, hdn;
  compare16(x, halo[3] >> 24, up, dn);
  compare16(halo, 0u, hup, hdn);  // only bits 2..15 are used (for lane 0's runs)
  u32 fav = ch.down_is_fav ? dn : up;
  u32 opp = ch.down_is_fav ? up : dn;
  const u32 hfav = readlane(ch.down_is_fav ? hdn : hup, 0);
  const u64 q0 = (u64)w * kDirectWin + 16 * lane;
  if (q0 == 0) {  // byte 0 has no predecessor
    fav &= ~1u;
    opp &= ~1u;
  }
  u32 keep = 0xFFFFu;  // bytes of the file
  if (q0 >= ch.n) keep = 0;
  else if (ch.n - q0 < 16) keep = (1u << (u32)(ch.n - q0)) - 1u;
  const u32 e = run_ends16(fav, shift_up_lanes(fav, hfav), ch.sl - 1) & keep;
  ch.E = e;
  ch.O = opp & keep;
  ch.cur = w;
  ch.emask = ballot(e != 0);
  ch.fe = e ? (u32)__builtin_ctz(e) : 16u;
  if (skipping(ch)) {
    const u32 cnt = (u32)__popc(ch.O);
    ch.incl = wave_incl_scan(cnt);
    ch.excl = ch.incl - cnt;
    ch.total = readlane(ch.incl, 63);
  }
}

// Group words: one lane's E or O bits.
__device__ __forceinline__ u32 read_group(u32 v, u32 g) { return readlane(v, g); }
__device__ __forceinline__ u64 read_group(u64 v, u32 g) { return readlane64(v, g); }
__device__ __forceinline__ u32 popcount(u32 v) { return (u32)__popc(v); }
__device__ __forceinline__ u32 popcount(u64 v) { return (u32)__popcll(v); }
__device__ __forceinline__ u32 lowest_bit(u32 v) { return (u32)__builtin_ctz(v); }
__device__ __forceinline__ u32 lowest_bit(u64 v) { return ctz64(v); }

template <u32 G>
struct GroupShift {
  static constexpr u32 value = G == 64 ? 6 : G == 16 ? 4 : 0;
  static_assert(value != 0, "groups are 16 or 64 bytes");
};

// Opposing pairs of the window at positions < pos (0 <= pos <= kWin).
template <class Ch>
__device__ __forceinline__ u32 opp_before(const Ch& ch, u32 pos) {
  typedef typename Ch::Word W;
  if (pos >= Ch::kWin) return ch.total;
  const u32 g = pos >> GroupShift<Ch::kG>::value, b = pos & (Ch::kG - 1);
  return readlane(ch.excl, g) + popcount(read_group(ch.O, g) & ~(~W(0) << b));  // the group's pairs below b
}

// First admissible run end of the current window at or after er (a byte
// offset in the window, possibly >= kWin), or kWin if none: in the word of
// group er/kG above er, else the first run end of the next group holding one
// (emask & (~1 << ge) are the groups after ge, none after the last).
template <class Ch>
__device__ __forceinline__ u32 first_end(const Ch& ch, u32 er) {
  typedef typename Ch::Word W;
  constexpr u32 kWin = Ch::kWin, kG = Ch::kG;
  if (er >= kWin) return kWin;
  const u32 ge = er >> GroupShift<kG>::value;
  const W word = read_group(ch.E, ge) & (~W(0) << (er & (kG - 1)));
  if (word) return ge * kG + lowest_bit(word);
  const u64 later = ch.emask & (~1ull << ge);
  if (!later) return kWin;
  const u32 g2 = ctz64(later);
  return g2 * kG + readlane(ch.fe, g2);
}

// Position in the current window of the need-th opposing pair at or after
// pr, or kWin if the window holds fewer (then *left = pairs it holds at or
// after pr).  The trigger is in the first group whose inclusive count
// reaches (pairs before pr) + need, at the right set bit of that group.
template <class Ch>
__device__ __forceinline__ u32 nth_opposing(const Ch& ch, u32 pr, u32 need, u32& left) {
  const u32 base = opp_before(ch, pr);
  left = ch.total - base;
  if (need > left) return Ch::kWin;
  const u32 target = base + need;
  const u32 gt = ctz64(ballot(ch.incl >= target));
  return gt * Ch::kG + select_bit((u64)read_group(ch.O, gt), target - readlane(ch.excl, gt));
}

// The cut that follows a cut (or a speculative start) at c.  Wave-uniform.
// Offsets inside the chunk are 32-bit, relative to c (max_size <= 1 GiB).
template <class Ch>
__device__ u64 next_cut(Ch& ch, u64 c) {
  constexpr u32 kWin = Ch::kWin;
  // rem = n - c, tested on its 32-bit halves (scalar compares): c >= n makes
  // it zero or wrap to a huge value (the top bit set, as streams are shorter
  // than 2^63 bytes)
  const u64 rem = ch.n - c;
  const u32 rem_hi = opaque_u32((u32)(rem >> 32)), rem_lo = opaque_u32((u32)rem);
  if (rem_hi >= 0x80000000u || (rem_hi == 0 && rem_lo == 0)) return ch.n;  // callers never ask past the end
  const u32 lim = (rem_hi != 0 || rem_lo > ch.max_size) ? ch.max_size : rem_lo;  // Sec. IV limit
  u32 s = ch.min_size - ch.sl;                                 // Sec. III-B scan start
  u32 p = s + 1;                                                    // next pair (p-1, p) to examine
  u32 need = ch.trig;                                               // opposing pairs still to the trigger
  const u32 c32 = (u32)c;
  for (;;) {
    if (p >= lim) return c + lim;
    if constexpr (Ch::kSummary) {
      // The last window entered held no run end (a stretch without run ends,
      // at the start of a chunk or when the scan leaves such a window): the
      // run-end summary tells whether any run end comes before the limit,
      // from the earliest admissible one on; if none, the chunk ends there.
      // Random data never asks.  One place, so its code is inlined once.
      if (ch.emask == 0 && ch.cur != kNone) {
        const u32 e_lo = s + ch.sl - 1;
        if (no_end_before(ch, (u32)((c + (e_lo > p ? e_lo : p)) >> 10), c + lim)) return c + lim;
      }
    }
    const u32 sub = (u32)((c + p) / kWin);
    ensure(ch, sub, (u32)((c + p + ch.min_size - ch.sl) / kWin));
    const u32 w = sub * kWin - c32;  // window start relative to c (mod 2^32)
    const u32 lw = lim - w < kWin ? lim - w : kWin;  // scan limit inside this window
    // events inside this window; a skip that lands in it continues here
    for (;;) {
      const u32 e_lo = s + ch.sl - 1;  // earliest admissible run end
      const u32 qe = first_end(ch, (e_lo > p ? e_lo : p) - w);
      u32 pt = kWin, left = 0;
      if (skipping(ch)) pt = nth_opposing(ch, p - w, need, left);
      if (qe < pt) {
        if (qe < lw) return c + (u32)(w + qe) + 1;  // Sec. III-A: boundary just past the run (w may wrap)
        return c + lim;                      // nothing before the limit
      }
      if (pt < kWin) {  // Sec. III-C: skip SkipSize bytes after the trigger byte
        if (pt >= lw) return c + lim;
        const u32 rel = w + pt + 1;  // just past the trigger, relative to c: rel <= lim as pt < lw
        if (ch.skip >= lim - rel) return c + lim;  // the scan would restart at or past the limit
        s = rel + ch.skip;
        p = s + 1;
        need = ch.trig;
        if (p - w < kWin) continue;  // the scan resumes in this window
        break;
      }
      need -= left;  // no event in this window
      p = w + kWin;
      if (p >= lim) return c + lim;
      break;
    }
  }
}

// ---------------------------------------------------------------------------
// Pass A and pass B
// ---------------------------------------------------------------------------

// Pass A of one chain: cuts from its segment start (taken as a cut) until the
// first cut at or past the segment end.  A single-segment file writes its
// output directly; otherwise the cuts, exit cut last, go to the chain's list.
template <class Ch>
__device__ __forceinline__ void run_pass_a(const FileDesc* __restrict__ files, const ChainWs& ws, u32 chain,
                                           SEQCDC_LOCAL u32x4* win) {
  const u32 lane = lane_id();
  const FileDesc& F = files[ws.chain_file[chain]];
  const u32 k = chain - F.chain0;
  const u64 S = (u64)k * F.seg;
  const u64 Send = (k + 1 == F.nseg) ? F.n : S + F.seg;
  const bool direct = F.nseg == 1;
  u64 cnt = 0;
  if (F.n) {
    Ch ch;
    chain_init(ch, F, win);
    SEQCDC_GLOBAL u64* dst = as_global(direct ? F.out : ws.list + ws.list_off[chain]);
    const u64 cap = direct ? F.out_cap : ~0ull;
    u64 buf = 0, c = S;
    do {
      c = next_cut(ch, c);
      if (lane == (u32)(cnt & 63)) buf = c;
      cnt++;
      if ((cnt & 63) == 0 || !before(c, Send)) {  // flush the lanes filled since the last flush
        const u64 i = ((cnt - 1) & ~63ull) + lane;
        if (i < cnt && i < cap) dst[i] = buf;
      }
    } while (before(c, Send));
  }
  if (lane == 0) {
    if (direct) *F.out_count = cnt;
    else ws.list_cnt[chain] = (u32)cnt;
  }
}

// Membership of x in the sorted main part (entries [0, cnt)) of a list,
// streaming forward (x must not decrease between calls on one cursor).
struct ListCursor {
  const u64* list;
  u32 cnt;
  u32 base;
  u64 vals;
  bool loaded;
};

__device__ __forceinline__ i32 cursor_find(ListCursor& lc, u64 x) {
  for (;;) {
    if (!lc.loaded) {
      const u32 i = lc.base + lane_id();
      lc.vals = i < lc.cnt ? as_global(lc.list)[i] : ~0ull;
      lc.loaded = true;
    }
    const u64 ge = ballot(lc.vals >= x);
    if (ge == 0) {
      if (lc.base + 64 < lc.cnt) {
        lc.base += 64;
        lc.loaded = false;
        continue;
      }
      return -1;
    }
    const u32 fl = ctz64(ge);
    return readlane64(lc.vals, fl) == x ? (i32)(lc.base + fl) : -1;
  }
}

constexpr u32 kOpen = 0xFFFFFFFFu;  // conv_chain of a continuation that stopped with its buffer full

// A continuation of `chain` (not the last of its file) from cut x, cc of its
// cuts already recorded: its cuts until one is also a cut of the chain that
// owns that position (or that chain's segment start), or the stream end.  Cut
// number i is stored at dst[i - base].  When cc reaches `stop` (pass B: the
// continuation's buffer is full) it stops and is left open at x, the next cut
// to examine: conv_chain = kOpen, conv_val = x.
template <class Ch>
__device__ void walk_continuation(const FileDesc& F, const ChainWs& ws, u32 chain, SEQCDC_LOCAL u32x4* win, u64 x,
                                  u64 cc, SEQCDC_GLOBAL u64* dst, u64 base, u64 stop) {
  const u64 n = F.n;
  const u32 nseg = F.nseg;
  u32 conv_chain = nseg;
  i32 conv_idx = -1;
  // Entries [from, cc) wait in the lanes (entry i in lane i % 64) and are
  // stored 64 at a time: a store per cut would make every later wait for a
  // window DMA wait for that store too (one counter covers loads and stores).
  const u32 lane = lane_id();
  u64 from = cc;
  u64 buf = 0;
  auto flush = [&]() {
    const u64 i = ((cc - 1) & ~63ull) + lane;
    if (cc > from && i >= from && i < cc) dst[i - base] = buf;
    from = cc;
  };
  if (x < n) {
    u32 m = (u32)min64(x / F.seg, nseg - 1);
    u64 Sm = (u64)m * F.seg;                          // start of chain m's segment
    u64 m_end = m + 1 < nseg ? Sm + F.seg : ~0ull;    // start of the next one (none after the last)
    Ch ch;
    chain_init(ch, F, win);
    ListCursor lc;
    auto open = [&](u32 seg) {
      const u32 cm = F.chain0 + seg;
      lc.list = ws.list + ws.list_off[cm];
      const u32 have = ws.list_cnt[cm];
      lc.cnt = have ? have - 1 : 0;  // main part: all but the exit cut
      lc.base = 0;
      lc.loaded = false;
    };
    open(m);
    for (;;) {
      const i32 idx = (x == Sm) ? -1 : cursor_find(lc, x);
      if (x == Sm || idx >= 0) {
        conv_chain = m;
        conv_idx = idx;
        break;
      }
      if (cc == stop) {
        conv_chain = kOpen;
        break;
      }
      const u64 nx = next_cut(ch, x);
      if (lane == (u32)(cc & 63)) buf = x;
      cc++;
      if ((cc & 63) == 0) flush();
      x = nx;
      if (x >= n) break;  // reached the end of the stream: conv_chain = nseg
      if (x >= m_end) {  // x moved into a later segment: min(x / seg, nseg - 1) > m
        m = (u32)min64(x / F.seg, nseg - 1);
        Sm = (u64)m * F.seg;
        m_end = m + 1 < nseg ? Sm + F.seg : ~0ull;
        open(m);
      }
    }
  }
  flush();
  if (lane == 0) {
    ws.conv_val[chain] = x;
    ws.conv_chain[chain] = conv_chain;
    ws.conv_idx[chain] = conv_idx;
    ws.cont_cnt[chain] = cc;
  }
}

// The exit cut of a multi-segment file's chain (the last entry of its list).
__device__ __forceinline__ u64 exit_cut(const ChainWs& ws, u32 chain) {
  const u32 cnt = ws.list_cnt[chain];
  return cnt ? ws.list[ws.list_off[chain] + cnt - 1] : ~0ull;
}

// Pass A over the chains in `order` (largest segments first), one wave per
// chain; waves take chains from an atomic counter, independently of the other
// waves of their workgroup.
// LDS window slots of one wave.
template <class Ch>
struct WaveLds;
template <>
struct WaveLds<MarkedChain> {
  static constexpr u32 kChunks = kRing * 64;
};
template <>
struct WaveLds<DirectChain> {
  static constexpr u32 kChunks = kDirectLdsChunks;
};

template <class Ch>
__global__ __launch_bounds__(256) void chains_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                     const u32* __restrict__ order, u32 nitems, u32* head) {
  __shared__ u32x4 win[kWavesPerGroup][WaveLds<Ch>::kChunks];
  SEQCDC_LOCAL u32x4* mine = (SEQCDC_LOCAL u32x4*)win[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
  for (;;) {
    const u32 t = wave_pop(head);
    if (t >= nitems) return;
    run_pass_a<Ch>(files, ws, order[t], mine);
  }
}

// Pass B over the chains in `order` (every chain but the last of each
// multi-segment file).
template <class Ch>
__global__ __launch_bounds__(256) void continue_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                       const u32* __restrict__ order, u32 nitems, u32* head) {
  __shared__ u32x4 win[kWavesPerGroup][WaveLds<Ch>::kChunks];
  SEQCDC_LOCAL u32x4* mine = (SEQCDC_LOCAL u32x4*)win[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
  for (;;) {
    const u32 t = wave_pop(head);
    if (t >= nitems) return;
    const u32 chain = order[t];
    walk_continuation<Ch>(files[ws.chain_file[chain]], ws, chain, mine, exit_cut(ws, chain), 0,
                          as_global(ws.cont + ws.cont_off[chain]), 0, ws.cont_cap);
  }
}

// Clears work counters and flags (grid-stride).
__global__ __launch_bounds__(256) void clear_kernel(u32* p, u64 count) {
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < count; i += (u64)gridDim.x * 256) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Stitch and compaction
// ---------------------------------------------------------------------------

constexpr u32 kStitchThreads = 1024;  // 16 waves
constexpr u32 kStitchWaves = kStitchThreads / 64;
constexpr u32 kStitchLdsRanges = 1024;  // covered ranges the stitch keeps in LDS (more go to global memory only)
constexpr u32 kStitchLdsJumps = 2048;   // jumps the stitch resolves in LDS in parallel (more: walked in order)

// Workgroup-wide exclusive scan of one 64-bit value per thread
// (kStitchThreads threads): a DPP scan inside each wave, then the wave totals
// through LDS.  Two barriers; *total receives the sum over the workgroup.
__device__ u64 block_exclusive_scan(u64 v, u64* sh, u64& total) {
  const u32 w = threadIdx.x >> 6;
  const u64 incl = wave_incl_scan64(v);
  if (lane_id() == 63) sh[w] = incl;
  __syncthreads();
  u64 pre = 0, tot = 0;
#pragma unroll
  for (u32 i = 0; i < kStitchWaves; i++) {
    const u64 x = sh[i];
    pre += i < w ? x : 0ull;
    tot += x;
  }
  total = tot;
  __syncthreads();  // sh is reused by the next scan
  return pre + incl - v;
}

// Stitch (one workgroup per multi-segment file): the exact cut sequence
// starts in chain 0 and moves to chain conv_chain[k] at conv_val[k].  Chains
// strictly between k and conv_chain[k] are covered by k's continuation and
// contribute nothing.  A continuation that stopped open (its buffer full, no
// convergence yet) covers, as far as is known, everything after it; if it is
// on the exact path, wave 0 continues it to its convergence (or the stream
// end), storing the further cuts in the file's overflow region, and the
// active chains are worked out again.  So the exact path is walked once, and
// continuations that turn out not to be on it are never taken further.
template <class Ch>
__global__ __launch_bounds__(kStitchThreads) void stitch_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                                const u32* __restrict__ multi, u32 nmulti) {
  __shared__ u32x4 swin[WaveLds<Ch>::kChunks];  // wave 0's window slots when it continues an open chain
  __shared__ u32 s_open;
  __shared__ u64 s_ovf_used;
  __shared__ u64 sh[kStitchWaves];
  __shared__ u32 scov[2 * kStitchLdsRanges];
  __shared__ u32 sjk[kStitchLdsJumps], sjn[kStitchLdsJumps];  // a jump's boundary and target chain
  __shared__ u32 snext[kStitchLdsJumps + 1], son[kStitchLdsJumps + 1];
  __shared__ u32 s_nj, s_nr;
  const u32 t = threadIdx.x;
  const FileDesc& F = files[multi[blockIdx.x]];
  const u32 nseg = F.nseg, c0 = F.chain0;
  uint2* jumps = (uint2*)(ws.jumps + 2 * (u64)c0);
  u32* cov = ws.covered + 2 * (u64)c0;
  if (t == 0) s_ovf_used = 0;

  for (;;) {  // rounds: once, plus once per open continuation on the exact path
  // 1. boundaries whose continuation skipped at least one whole segment,
  // with the chain each one ends in (an open one: the end, nseg)
  u32 base = 0;
  for (u32 j0 = 0; j0 < nseg; j0 += kStitchThreads) {
    const u32 k = j0 + t;
    u32 nx = k + 1 < nseg ? ws.conv_chain[c0 + k] : 0u;
    if (nx == kOpen) nx = nseg;
    const bool jump = k + 1 < nseg && nx != k + 1;
    u64 tot;
    const u32 pos = (u32)block_exclusive_scan(jump ? 1u : 0u, sh, tot);
    if (jump) {
      jumps[base + pos] = make_uint2(k, nx);
      if (base + pos < kStitchLdsJumps) {
        sjk[base + pos] = k;
        sjn[base + pos] = nx;
      }
    }
    base += (u32)tot;
  }
  if (t == 0) s_nj = base;
  __syncthreads();

  // 2. the active jumps: a jump from an active chain covers (k, next), and
  // the first jump is active.  In order, the next active jump after jump i
  // is the first later one whose boundary its range does not cover, its
  // successor.  The active jumps are the successors of jump 0, repeatedly.
  const u32 nj = s_nj;
  u32 nr = 0;
  if (nj <= kStitchLdsJumps) {
    // In LDS, in parallel: each jump's successor by binary search over the
    // boundaries (increasing), then the jumps reachable from jump 0 by pointer
    // doubling, then the ranges of the marked jumps in order by a scan.
    // Index nj stands for "no successor".
    for (u32 i = t; i < nj; i += kStitchThreads) {
      const u32 target = sjn[i];
      u32 lo = i + 1, hi = nj;  // first later jump with boundary >= target
      while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (sjk[mid] < target) lo = mid + 1;
        else hi = mid;
      }
      snext[i] = lo;
      son[i] = i == 0 ? 1u : 0u;
    }
    if (t == 0) {
      snext[nj] = nj;
      son[nj] = 0u;
    }
    __syncthreads();
    // after the round with step 2^r, every jump within 2^(r+1) - 1 successors
    // of jump 0 is marked (and only such jumps: marks only follow successors)
    for (u32 step = 1; step < nj; step <<= 1) {
      u32 nv[kStitchLdsJumps / kStitchThreads];
#pragma unroll
      for (u32 q = 0; q < kStitchLdsJumps / kStitchThreads; q++) {
        const u32 i = t + q * kStitchThreads;
        nv[q] = i < nj ? snext[i] : nj;
        if (i < nj && son[i]) son[nv[q]] = 1u;
      }
      __syncthreads();
      u32 n2[kStitchLdsJumps / kStitchThreads];
#pragma unroll
      for (u32 q = 0; q < kStitchLdsJumps / kStitchThreads; q++) n2[q] = snext[nv[q]];
      __syncthreads();
#pragma unroll
      for (u32 q = 0; q < kStitchLdsJumps / kStitchThreads; q++) {
        const u32 i = t + q * kStitchThreads;
        if (i < nj) snext[i] = n2[q];
      }
      __syncthreads();
    }
    for (u32 j0 = 0; j0 < nj; j0 += kStitchThreads) {
      const u32 i = j0 + t;
      const bool act = i < nj && son[i] != 0u;
      u64 tot;
      const u32 pos = nr + (u32)block_exclusive_scan(act ? 1u : 0u, sh, tot);
      if (act) {
        cov[2 * pos] = sjk[i] + 1;
        cov[2 * pos + 1] = sjn[i];  // covered: k+1 .. nx-1
        if (pos < kStitchLdsRanges) {
          scov[2 * pos] = sjk[i] + 1;
          scov[2 * pos + 1] = sjn[i];
        }
      }
      nr += (u32)tot;
    }
  } else if (t < 64) {
    // Too many for LDS: wave 0 walks them in order, 64 at a time from its
    // lanes, going from one active jump straight to the next by ballot.
    u32 until = 0, wn = 0;
    for (u32 i0 = 0; i0 < nj; i0 += 64) {
      const bool valid = i0 + t < nj;
      const uint2 jv = valid ? jumps[i0 + t] : make_uint2(0u, 0u);
      u64 left = ballot(valid);  // lanes not walked past yet
      for (;;) {
        const u64 cand = left & ballot(jv.x >= until);  // k >= until: k itself is not covered
        if (!cand) break;
        const u32 q = ctz64(cand);
        left = q < 63 ? left & (~0ull << (q + 1)) : 0ull;
        const u32 k = readlane(jv.x, q);
        const u32 nx = readlane(jv.y, q);
        if (t == 0) {
          cov[2 * wn] = k + 1;
          cov[2 * wn + 1] = nx;  // covered: k+1 .. nx-1
          if (wn < kStitchLdsRanges) {
            scov[2 * wn] = k + 1;
            scov[2 * wn + 1] = nx;
          }
        }
        wn++;
        until = nx;
      }
    }
    if (t == 0) s_nr = wn;
  }
  __syncthreads();
  if (nj > kStitchLdsJumps) nr = s_nr;
  const bool in_lds = nr <= kStitchLdsRanges;

  // 3. active flags; 4. entry index of each active chain
  for (u32 j = t; j < nseg; j += kStitchThreads) {
    u32 lo = 0, hi = nr;  // first range with start > j
    while (lo < hi) {
      u32 mid = (lo + hi) >> 1;
      if ((in_lds ? scov[2 * mid] : cov[2 * mid]) <= j) lo = mid + 1;
      else hi = mid;
    }
    const bool covered = lo > 0 && j < (in_lds ? scov[2 * (lo - 1) + 1] : cov[2 * (lo - 1) + 1]);
    ws.active[c0 + j] = covered ? 0u : 1u;
    if (j == 0) ws.entry_idx[c0] = 0;
  }
  if (t == 0) s_open = nseg;
  __syncthreads();
  // the first open continuation on the exact path, if any
  for (u32 k = t; k + 1 < nseg; k += kStitchThreads)
    if (ws.active[c0 + k] && ws.conv_chain[c0 + k] == kOpen) atomicMin(&s_open, k);
  __syncthreads();
  const u32 ko = s_open;
  if (ko >= nseg) break;
  if (t < 64) {  // wave 0 continues it; its further cuts go to the file's overflow region
    const u32 chain = c0 + ko;
    const u64 cc = ws.cont_cnt[chain];  // = cont_cap: the buffer is full
    const u64 at = F.ovf0 + s_ovf_used;
    walk_continuation<Ch>(F, ws, chain, (SEQCDC_LOCAL u32x4*)swin, ws.conv_val[chain], cc, as_global(ws.ovf + at), cc,
                          ~0ull);
    if (t == 0) {
      ws.ovf_start[chain] = at;
      s_ovf_used += ws.cont_cnt[chain] - cc;
    }
  }
  __threadfence_block();
  __syncthreads();
  }  // rounds
  for (u32 k = t; k + 1 < nseg; k += kStitchThreads) {
    if (!ws.active[c0 + k]) continue;
    const u32 nx = ws.conv_chain[c0 + k];
    if (nx < nseg) ws.entry_idx[c0 + nx] = ws.conv_idx[c0 + k];
  }
  __syncthreads();

  // 5. output count of each chain; 6. offsets
  u64 obase = 0;
  for (u32 j0 = 0; j0 < nseg; j0 += kStitchThreads) {
    const u32 j = j0 + t;
    u64 cnt = 0;
    if (j < nseg && ws.active[c0 + j]) {
      const i32 e = ws.entry_idx[c0 + j];
      const u64 main_cnt = ws.list_cnt[c0 + j] - 1;
      const bool last = j + 1 == nseg;
      cnt = (j > 0 && e < 0 ? 1 : 0) + (main_cnt - (u64)(e > 0 ? e : 0));
      if (!last) cnt += ws.cont_cnt[c0 + j];
      if (last || ws.conv_chain[c0 + j] == nseg) cnt += 1;  // the stream end
    }
    u64 tot;
    const u64 pos = block_exclusive_scan(cnt, sh, tot);
    if (j < nseg) ws.out_off[c0 + j] = obase + pos;
    obase += tot;
  }
  if (t == 0) *F.out_count = obase;
}

// Compaction: one wave per chain of a multi-segment file copies its exact
// part: the main part of its list, its continuation buffer and, for a
// continuation the stitch took further, its overflow cuts.
__global__ __launch_bounds__(256) void compact_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                      const u32* __restrict__ chains, u32 nchains) {
  const u32 lane = lane_id();
  const u32 w = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6));  // wave-uniform
  if (w >= nchains) return;
  const u32 chain = chains[w];
  if (!ws.active[chain]) return;
  const FileDesc& F = files[ws.chain_file[chain]];
  const u32 j = chain - F.chain0;
  const bool last = j + 1 == F.nseg;
  u64* out = F.out;
  const u64 cap = F.out_cap;
  u64 o = ws.out_off[chain];
  const i32 e = ws.entry_idx[chain];
  if (j > 0 && e < 0) {
    if (lane == 0 && o < cap) out[o] = (u64)j * F.seg;
    o++;
  }
  const u64* list = ws.list + ws.list_off[chain];
  const u64 main_cnt = ws.list_cnt[chain] - 1;
  for (u64 i = (u64)(e > 0 ? e : 0); i < main_cnt; i += 64) {
    const u64 ii = i + lane;
    if (ii < main_cnt && o + (ii - i) < cap) out[o + (ii - i)] = list[ii];
    o += (main_cnt - i < 64) ? main_cnt - i : 64;
  }
  if (!last) {
    const u64 cc = ws.cont_cnt[chain];
    const u64 stored = cc < ws.cont_cap ? cc : ws.cont_cap;
    const u64* cont = ws.cont + ws.cont_off[chain];
    for (u64 i = 0; i < stored; i += 64) {
      const u64 ii = i + lane;
      if (ii < stored && o + (ii - i) < cap) out[o + (ii - i)] = cont[ii];
      o += (stored - i < 64) ? stored - i : 64;
    }
    const u64 extra = cc - stored;  // cuts the stitch added after the buffer filled
    const u64* ovf = ws.ovf + (extra ? ws.ovf_start[chain] : 0);
    for (u64 i = 0; i < extra; i += 64) {
      const u64 ii = i + lane;
      if (ii < extra && o + (ii - i) < cap) out[o + (ii - i)] = ovf[ii];
      o += (extra - i < 64) ? extra - i : 64;
    }
  }
  if (last || ws.conv_chain[chain] == F.nseg) {
    if (lane == 0 && o < cap) out[o] = F.n;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_clear(u32* p, u64 count, hipStream_t st) {
  const u64 groups = (count + 255) / 256;
  hipLaunchKernelGGL(clear_kernel, dim3((u32)(groups < 1024 ? (groups ? groups : 1) : 1024)), dim3(256), 0, st, p,
                     count);
  return hipGetLastError();
}

hipError_t launch_chains(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32* head,
                         u32 groups, bool direct, hipStream_t st) {
  if (!nitems) return hipSuccess;
  if (direct)
    hipLaunchKernelGGL(chains_kernel<DirectChain>, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems, head);
  else
    hipLaunchKernelGGL(chains_kernel<MarkedChain>, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems, head);
  return hipGetLastError();
}

hipError_t launch_continue(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32* head,
                           u32 groups, bool direct, hipStream_t st) {
  if (!nitems) return hipSuccess;
  if (direct)
    hipLaunchKernelGGL(continue_kernel<DirectChain>, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems,
                       head);
  else
    hipLaunchKernelGGL(continue_kernel<MarkedChain>, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems,
                       head);
  return hipGetLastError();
}

hipError_t launch_stitch(const FileDesc* d_files, const ChainWs& ws, const u32* d_multi, u32 nmulti, bool direct,
                         hipStream_t st) {
  if (!nmulti) return hipSuccess;
  if (direct)
    hipLaunchKernelGGL(stitch_kernel<DirectChain>, dim3(nmulti), dim3(kStitchThreads), 0, st, d_files, ws, d_multi,
                       nmulti);
  else
    hipLaunchKernelGGL(stitch_kernel<MarkedChain>, dim3(nmulti), dim3(kStitchThreads), 0, st, d_files, ws, d_multi,
                       nmulti);
  return hipGetLastError();
}

hipError_t launch_compact(const FileDesc* d_files, const ChainWs& ws, const u32* d_chains, u32 nchains,
                          hipStream_t st) {
  if (!nchains) return hipSuccess;
  const u32 groups = (nchains + kWavesPerGroup - 1) / kWavesPerGroup;
  hipLaunchKernelGGL(compact_kernel, dim3(groups), dim3(256), 0, st, d_files, ws, d_chains, nchains);
  return hipGetLastError();
}

}  // namespace seqcdc
