// SeqCDC chunk-boundary detection on CDNA4 (gfx950).
//
// The method (Udayashankar & Al-Kiswany, arXiv 2505.21194): a chunk ends
// right after the first run of SeqLength strictly monotone bytes (Sec.
// III-A) found at or after min - SeqLength bytes into the chunk (Sec.
// III-B); after SkipTrigger opposing pairs the next SkipSize bytes are not
// scanned and the counters restart (Sec. III-C); a chunk never exceeds the
// maximum size (Sec. IV).
//
// Two phases, as in the vector formulation of Sec. III-D:
//   mark    - bandwidth-bound: every byte pair becomes one favourable bit F,
//             one opposing bit O; E = AND of SeqLength-1 shifted F masks marks
//             the bytes that end a candidate run.  Written packed (EO16).
//   resolve - the exact sequential state machine over E/O with ballots,
//             ctz, popcount and a select-n-th-bit, run speculatively from
//             every segment start (chains), followed by a convergence pass
//             (continuations), a stitch that picks the exact pieces and a
//             compaction into the caller's cut list.
// Cut positions are exclusive chunk ends; the last one is the stream length.

#include <hip/hip_runtime.h>

#include "seqcdc_internal.h"

namespace seqcdc {

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u32 lane_id() { return __lane_id(); }

// lane l receives v of lane l-1; lane 0 receives `carry` (DPP wave_shr:1).
__device__ __forceinline__ u32 shift_up_lanes(u32 v, u32 carry) {
  return __builtin_amdgcn_update_dpp(carry, v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ u32 readlane(u32 v, u32 l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ u64 readlane64(u64 v, u32 l) {
  return (u64)readlane((u32)v, l) | ((u64)readlane((u32)(v >> 32), l) << 32);
}
__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ u32 ctz64(u64 v) { return (u32)__builtin_ctzll(v); }

// Inclusive prefix sum across the wave (DPP row shifts + row broadcasts).
__device__ __forceinline__ u32 wave_incl_scan(u32 v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false); // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false); // row_bcast:31
  return v;
}

// ---------------------------------------------------------------------------
// Mark
// ---------------------------------------------------------------------------

// Per-halfword unsigned difference; bit 15 / bit 31 is set iff a < b.
__device__ __forceinline__ u32 sub16x2(u32 a, u32 b) {
  us2 va = __builtin_bit_cast(us2, a), vb = __builtin_bit_cast(us2, b);
  return __builtin_bit_cast(u32, (us2)(va - vb));
}

// Four 0x00/0xFF byte masks (one dword per 4 input bytes, in byte order) ->
// 16 bits, bit i = byte i.
__device__ __forceinline__ u32 pack16(u32 m0, u32 m1, u32 m2, u32 m3) {
  const u32 sel = 0x88442211u;  // byte j keeps bit j (from the low dword) and bit 4+j (high dword)
  u32 t01 = ((m0 & 0x0F0F0F0Fu) | (m1 & 0xF0F0F0F0u)) & sel;
  u32 t23 = ((m2 & 0x0F0F0F0Fu) | (m3 & 0xF0F0F0F0u)) & sel;
  u32 hi = __builtin_amdgcn_sad_u8(t23, 0u, 0u);  // sum of bytes = OR of disjoint bits
  return __builtin_amdgcn_sad_u8(t01, 0u, hi << 8);
}

// For the 16 bytes x[0..3] (little endian) preceded by byte `prev`:
// up16 bit i = byte i > its predecessor, down16 bit i = byte i < its predecessor.
__device__ __forceinline__ void compare16(const u32 x[4], u32 prev, u32& up16, u32& down16) {
  u32 mu[4], md[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    u32 before = k ? x[k - 1] : (prev << 24);
    u32 xe = x[k] & 0x00FF00FFu;                                   // bytes 0, 2
    u32 xo = (x[k] >> 8) & 0x00FF00FFu;                            // bytes 1, 3
    u32 pe = __builtin_amdgcn_perm(x[k], before, 0x0c050c03u);     // predecessors of bytes 0, 2
    // predecessors of bytes 1, 3 are bytes 0, 2 (= xe)
    u32 up_e = sub16x2(pe, xe), up_o = sub16x2(xe, xo);
    u32 dn_e = sub16x2(xe, pe), dn_o = sub16x2(xo, xe);
    // gather the four sign bits in byte order as 0x00/0xFF bytes
    mu[k] = __builtin_amdgcn_perm(up_o, up_e, 0x0B090A08u);
    md[k] = __builtin_amdgcn_perm(dn_o, dn_e, 0x0B090A08u);
  }
  up16 = pack16(mu[0], mu[1], mu[2], mu[3]);
  down16 = pack16(md[0], md[1], md[2], md[3]);
}

// Bits 16..31 of the AND of (len) consecutive bits ending at each position of
// ext = (cur16 << 16) | prev16, i.e. which of the 16 current bytes end a run of
// `len` favourable pairs.
__device__ __forceinline__ u32 run_ends16(u32 cur16, u32 prev16, u32 len) {
  u32 r = (cur16 << 16) | prev16;
  u32 have = 1;
  while (have < len) {
    u32 sh = have < len - have ? have : len - have;
    r &= r << sh;
    have += sh;
  }
  return r >> 16;
}

// 16 bytes starting `r` (0..15) bytes into the aligned 32 bytes (lo, hi).
__device__ __forceinline__ void funnel16(const uint4& lo, const uint4& hi, u32 r, u32 x[4]) {
  u32 d[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  u32 a = r >> 2, b = r & 3;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    u32 w0 = d[k], w1 = d[k + 1], w2 = d[k + 2], w3 = d[k + 3], w4 = d[k + 4];
    u32 l0 = a == 0 ? w0 : a == 1 ? w1 : a == 2 ? w2 : w3;
    u32 l1 = a == 0 ? w1 : a == 1 ? w2 : a == 2 ? w3 : w4;
    x[k] = __builtin_amdgcn_alignbyte(l1, l0, b);
  }
}

// Load the 16 bytes of this lane for the 1 KiB block at file offset B.  All
// loads are 16-byte aligned: a 16-byte aligned chunk never straddles a page,
// so chunks that overlap the stream [data, data+n) are safe to read whole;
// bytes outside the stream are ignored by the caller.
__device__ __forceinline__ void load_block(const uint8_t* data, u64 n, u64 B, u32 x[4]) {
  const u32 lane = lane_id();
  const uintptr_t addr = (uintptr_t)data;
  const u32 r = (u32)(addr & 15);
  const uint4* base = (const uint4*)(addr - r);  // aligned view; byte q of the stream is at r + q
  const u64 first = (B >> 4) + lane;              // aligned chunk index of this lane
  const u64 end_chunk = (r + n + 15) >> 4;        // aligned chunks overlapping the stream
  uint4 lo = make_uint4(0, 0, 0, 0);
  if (first < end_chunk) {
    u32x4 v = __builtin_nontemporal_load((const u32x4*)(base + first));
    lo = make_uint4(v.x, v.y, v.z, v.w);
  }
  if (r == 0) {
    x[0] = lo.x; x[1] = lo.y; x[2] = lo.z; x[3] = lo.w;
    return;
  }
  uint4 hi;
  hi.x = __shfl_down(lo.x, 1);
  hi.y = __shfl_down(lo.y, 1);
  hi.z = __shfl_down(lo.z, 1);
  hi.w = __shfl_down(lo.w, 1);
  if (lane == 63) {
    hi = make_uint4(0, 0, 0, 0);
    if (first + 1 < end_chunk) hi = base[first + 1];
  }
  funnel16(lo, hi, r, x);
}

// 16 bytes at file offset B-16 (B >= 16) for the halo, wave-uniform.
__device__ __forceinline__ void load_halo(const uint8_t* data, u64 n, u64 B, u32 x[4]) {
  const uintptr_t addr = (uintptr_t)data;
  const u32 r = (u32)(addr & 15);
  const uint4* base = (const uint4*)(addr - r);
  const u64 c0 = (B - 16) >> 4;
  uint4 lo = base[c0];
  if (r == 0) {
    x[0] = lo.x; x[1] = lo.y; x[2] = lo.z; x[3] = lo.w;
    return;
  }
  uint4 hi = base[c0 + 1];  // overlaps byte B-1 < n, so it overlaps the stream
  funnel16(lo, hi, r, x);
}

// One wave marks `U` consecutive 1 KiB blocks of one file.  Files are located
// by a binary search over their first mark span.
template <int U>
__global__ __launch_bounds__(256) void mark_kernel(const FileDesc* __restrict__ files, u32 nfiles, u64 total_spans,
                                                   u32* __restrict__ counters) {
  const u32 lane = lane_id();
  const u64 span = (u64)blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x < 2) counters[threadIdx.x] = 0;  // queue heads of the resolve kernels
  if (span >= total_spans) return;
  u32 lo = 0, hi = nfiles;
  while (hi - lo > 1) {
    u32 mid = (lo + hi) >> 1;
    if (files[mid].mark_span0 <= span) lo = mid;
    else hi = mid;
  }
  const FileDesc& F = files[lo];
  const uint8_t* data = F.data;
  const u64 n = F.n;
  const u32 down_is_fav = F.mode;  // decreasing mode: favourable = byte below its predecessor
  const u32 runlen = F.sl - 1;
  u32* __restrict__ eo = F.eo;
  const u64 nblk = (n + kMarkBlock - 1) / kMarkBlock;
  u64 blk = (span - F.mark_span0) * U;

  u32 carry_byte = 0, carry_fav = 0;  // last byte / F bits of the 16 bytes before the block
  if (blk > 0) {
    u32 h[4];
    load_halo(data, n, blk * kMarkBlock, h);
    u32 up, dn;
    compare16(h, 0u, up, dn);  // bit 0 is wrong (unknown predecessor) but is never used for SeqLength <= 16
    carry_fav = down_is_fav ? dn : up;
    carry_byte = h[3] >> 24;
  }

#pragma unroll 1
  for (int u = 0; u < U; u++, blk++) {
    if (blk >= nblk) break;
    const u64 B = blk * kMarkBlock;
    u32 x[4];
    load_block(data, n, B, x);
    const u32 last = x[3] >> 24;
    const u32 prev = shift_up_lanes(last, carry_byte);
    u32 up, dn;
    compare16(x, prev, up, dn);
    u32 fav = down_is_fav ? dn : up;
    u32 opp = down_is_fav ? up : dn;
    if (B == 0 && lane == 0) {  // byte 0 has no predecessor
      fav &= ~1u;
      opp &= ~1u;
    }
    const u32 fav_prev = shift_up_lanes(fav, carry_fav);
    u32 e = run_ends16(fav, fav_prev, runlen);
    const u64 q0 = B + 16ull * lane;
    bool store = true;
    if (B + kMarkBlock > n) {  // tail block: clear bits of bytes >= n
      if (q0 >= n) {
        e = opp = 0;
        store = q0 < ((n + 63) & ~63ull);
      } else if (n - q0 < 16) {
        u32 keep = (1u << (u32)(n - q0)) - 1u;
        e &= keep;
        opp &= keep;
      }
    }
    if (store) eo[(B >> 4) + lane] = e | (opp << 16);
    carry_byte = readlane(last, 63);
    carry_fav = readlane(fav, 63);
  }
}

// ---------------------------------------------------------------------------
// Resolve: the sequential state machine over E/O
// ---------------------------------------------------------------------------

struct Chain {
  const uint4* eo;
  u64 n, groups;
  u64 min_size, max_size;
  u32 sl, trig, skip;
  // current window: lane l holds group wb + l
  u64 wb;
  u64 E, O;
  bool have;
};

__device__ __forceinline__ void chain_init(Chain& ch, const FileDesc& F) {
  ch.eo = (const uint4*)F.eo;
  ch.n = F.n;
  ch.groups = (F.n + 63) >> 6;
  ch.min_size = F.min_size;
  ch.max_size = F.max_size;
  ch.sl = F.sl;
  ch.trig = F.trig;
  ch.skip = F.skip;
  ch.have = false;
  ch.wb = 0;
  ch.E = ch.O = 0;
}

__device__ __forceinline__ void load_window(Chain& ch, u64 wb) {
  const u64 g = wb + lane_id();
  u64 E = 0, O = 0;
  if (g < ch.groups) {
    uint4 v = ch.eo[g];
    E = (u64)__builtin_amdgcn_perm(v.y, v.x, 0x05040100u) | ((u64)__builtin_amdgcn_perm(v.w, v.z, 0x05040100u) << 32);
    O = (u64)__builtin_amdgcn_perm(v.y, v.x, 0x07060302u) | ((u64)__builtin_amdgcn_perm(v.w, v.z, 0x07060302u) << 32);
  }
  ch.E = E;
  ch.O = O;
  ch.wb = wb;
  ch.have = true;
}

// Bits of the 64 bytes starting at P that lie in [lo, hi] (inclusive).
__device__ __forceinline__ u64 range_bits(u64 P, u64 lo, u64 hi) {
  if (lo > hi || hi < P || lo > P + 63) return 0;
  u64 m = ~0ull;
  if (lo > P) m <<= (u32)(lo - P);
  if (hi < P + 63) m &= ~0ull >> (u32)(63 - (hi - P));
  return m;
}

// Position of the k-th (1-based) set bit of the wave-uniform word w.
__device__ __forceinline__ u32 select_kth(u64 w, u32 k) {
  const u32 lane = lane_id();
  u32 below = __builtin_amdgcn_mbcnt_hi((u32)(w >> 32), __builtin_amdgcn_mbcnt_lo((u32)w, 0u));
  bool set = (w >> lane) & 1ull;
  return ctz64(ballot(set && below == k - 1));
}

// The cut that follows a cut (or stream start) at c.  Wave-uniform.
__device__ u64 next_cut(Chain& ch, u64 c) {
  const u64 n = ch.n;
  const u64 L = (n - c > ch.max_size) ? c + ch.max_size : n;  // Sec. IV limit
  u64 s = c + ch.min_size - ch.sl;                            // Sec. III-B scan start
  u64 p = s + 1;                                              // first pair (p-1, p) to examine
  u64 e_lo = s + ch.sl - 1;                                   // earliest admissible run end
  u32 ocnt = 0;                                               // opposing pairs since s
  const bool skipping = ch.trig != kNoSkip;
  for (;;) {
    if (p >= L) return L;
    const u64 g = p >> 6;
    if (!ch.have || g < ch.wb || g >= ch.wb + 64) load_window(ch, g);
    const u64 P = (ch.wb + lane_id()) << 6;
    const u64 hi = L - 1;
    const u64 Em = ch.E & range_bits(P, e_lo > p ? e_lo : p, hi);
    const u64 Om = ch.O & range_bits(P, p, hi);
    u64 qe = ~0ull, qt = ~0ull;
    const u64 eb = ballot(Em != 0);
    if (eb) {
      const u32 le = ctz64(eb);
      qe = ((ch.wb + le) << 6) + ctz64(readlane64(Em, le));
    }
    u32 total = 0;
    if (skipping) {
      const u32 cnt = (u32)__popcll(Om);
      const u32 incl = wave_incl_scan(cnt);
      total = readlane(incl, 63);
      const u32 need = ch.trig - ocnt;
      if (total >= need) {
        const u32 lt = ctz64(ballot(incl >= need));
        const u32 before = readlane(incl - cnt, lt);
        qt = ((ch.wb + lt) << 6) + select_kth(readlane64(Om, lt), need - before);
      }
    }
    if (qe < qt) return qe + 1;  // Sec. III-A: boundary just past the run
    if (qt != ~0ull) {           // Sec. III-C: skip SkipSize bytes after the trigger byte
      s = qt + 1 + ch.skip;
      p = s + 1;
      e_lo = s + ch.sl - 1;
      ocnt = 0;
      continue;
    }
    ocnt += total;
    p = (ch.wb + 64) << 6;
  }
}

__device__ __forceinline__ u32 wave_pop(u32* head) {
  u32 v = 0;
  if (lane_id() == 0) v = atomicAdd(head, 1u);
  return __builtin_amdgcn_readfirstlane(v);
}

// Pass A: each chain starts at its segment start as if a cut were there and
// records every cut up to and including the first one at or past the segment
// end (its exit).  Chains of single-segment files write the final output.
__global__ __launch_bounds__(256) void chains_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                     const u32* __restrict__ order, u32 nitems) {
  const u32 lane = lane_id();
  for (;;) {
    const u32 it = wave_pop(&ws.counters[0]);
    if (it >= nitems) return;
    const u32 chain = order[it];
    const u32 f = ws.chain_file[chain];
    const FileDesc& F = files[f];
    if (F.n == 0) {
      if (lane == 0) *F.out_count = 0;
      continue;
    }
    const u32 k = chain - F.chain0;
    const u64 S = (u64)k * F.seg;
    const u64 Send = (k + 1 == F.nseg) ? F.n : S + F.seg;
    Chain ch;
    chain_init(ch, F);
    const bool direct = F.nseg == 1;
    u64* dst = direct ? F.out : ws.list + ws.list_off[chain];
    const u64 cap = direct ? F.out_cap : ~0ull;
    u64 cnt = 0, c = S;
    u64 buf = 0;
    do {
      c = next_cut(ch, c);
      if (lane == (u32)(cnt & 63)) buf = c;
      cnt++;
      if ((cnt & 63) == 0 || c >= Send) {  // flush the lanes filled since the last flush
        const u64 base = (cnt - 1) & ~63ull;
        const u64 i = base + lane;
        if (i < cnt && i < cap) dst[i] = buf;
      }
    } while (c < Send);
    if (lane == 0) {
      if (direct) *F.out_count = cnt;
      else ws.list_cnt[chain] = (u32)cnt;
    }
  }
}

// Membership of x in the sorted main part (entries [0, cnt)) of a list,
// streaming forward from `base` (wave-uniform state kept by the caller).
struct ListCursor {
  const u64* list;
  u32 cnt;
  u32 base;
  u64 vals;
  bool loaded;
};

__device__ __forceinline__ void cursor_load(ListCursor& lc) {
  const u32 i = lc.base + lane_id();
  lc.vals = i < lc.cnt ? lc.list[i] : ~0ull;
  lc.loaded = true;
}

// Returns the index of x in the list, or -1 if absent.  x must not decrease
// between calls on one cursor.
__device__ __forceinline__ i32 cursor_find(ListCursor& lc, u64 x) {
  for (;;) {
    if (!lc.loaded) cursor_load(lc);
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

// Pass B: continue chain k from its exit cut until one of its cuts is also a
// cut of the chain that owns that position (or the start of its segment).
// From that shared cut on, both chains are the same sequence: the state after
// a cut depends only on the cut position.
__global__ __launch_bounds__(256) void continue_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                       const u32* __restrict__ order, u32 nitems) {
  const u32 lane = lane_id();
  for (;;) {
    const u32 it = wave_pop(&ws.counters[1]);
    if (it >= nitems) return;
    const u32 chain = order[it];
    const FileDesc& F = files[ws.chain_file[chain]];
    const u64 n = F.n;
    const u32 nseg = F.nseg;
    u64 x = ws.list[ws.list_off[chain] + ws.list_cnt[chain] - 1];
    u32 conv_chain = nseg;
    i32 conv_idx = -1;
    u32 cc = 0;
    u64* cont = ws.cont + ws.cont_off[chain];
    if (x < n) {
      Chain ch;
      chain_init(ch, F);
      u32 m = (u32)(x / F.seg);
      if (m >= nseg) m = nseg - 1;
      ListCursor lc;
      auto open = [&](u32 seg) {
        const u32 cm = F.chain0 + seg;
        lc.list = ws.list + ws.list_off[cm];
        lc.cnt = ws.list_cnt[cm] - 1;  // main part: all but the exit cut
        lc.base = 0;
        lc.loaded = false;
      };
      open(m);
      for (;;) {
        const u64 Sm = (u64)m * F.seg;
        const i32 idx = (x == Sm) ? -1 : cursor_find(lc, x);
        if (x == Sm || idx >= 0) {
          conv_chain = m;
          conv_idx = idx;
          break;
        }
        if (lane == 0 && cc < ws.cont_cap) cont[cc] = x;
        cc++;
        x = next_cut(ch, x);
        if (x >= n) break;  // reached the end of the stream: conv_chain = nseg
        u32 m2 = (u32)(x / F.seg);
        if (m2 >= nseg) m2 = nseg - 1;
        if (m2 != m) {
          m = m2;
          open(m);
        }
      }
    }
    if (lane == 0) {
      ws.conv_val[chain] = x;
      ws.conv_chain[chain] = conv_chain;
      ws.conv_idx[chain] = conv_idx;
      ws.cont_cnt[chain] = cc;
    }
  }
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ u64 block_exclusive_scan(u64 v, u64* sh, u64& total) {
  const u32 t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (u32 d = 1; d < 256; d <<= 1) {
    u64 a = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[255];
  u64 r = sh[t] - v;
  __syncthreads();
  return r;
}

// Stitch (one 256-thread workgroup per multi-segment file): the exact cut
// sequence starts in chain 0 and moves to chain conv_chain[k] at conv_val[k].
// Chains strictly between k and conv_chain[k] are covered by k's
// continuation and contribute nothing.
__global__ __launch_bounds__(256) void stitch_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                     const u32* __restrict__ multi, u32 nmulti) {
  __shared__ u64 sh[256];
  __shared__ u32 s_nj, s_nr;
  const u32 t = threadIdx.x;
  const FileDesc& F = files[multi[blockIdx.x]];
  const u32 nseg = F.nseg, c0 = F.chain0;
  u32* jumps = ws.jumps + c0;
  u32* cov = ws.covered + 2 * (u64)c0;

  // 1. boundaries whose continuation skipped at least one whole segment
  u64 base = 0;
  for (u32 j0 = 0; j0 < nseg; j0 += 256) {
    const u32 k = j0 + t;
    const bool jump = k + 1 < nseg && ws.conv_chain[c0 + k] != k + 1;
    u64 tot;
    const u64 pos = block_exclusive_scan(jump ? 1 : 0, sh, tot);
    if (jump) jumps[base + pos] = k;
    base += tot;
  }
  if (t == 0) s_nj = (u32)base;
  __syncthreads();

  // 2. walk the jumps in order; a jump from an active chain covers (k, next)
  if (t == 0) {
    u32 until = 0, nr = 0;
    for (u32 i = 0; i < s_nj; i++) {
      const u32 k = jumps[i];
      if (k < until) continue;  // k itself is covered
      const u32 nx = ws.conv_chain[c0 + k];
      cov[2 * nr] = k + 1;
      cov[2 * nr + 1] = nx;  // covered: k+1 .. nx-1
      nr++;
      until = nx;
    }
    s_nr = nr;
  }
  __syncthreads();
  const u32 nr = s_nr;

  // 3. active flags; 4. entry index of each active chain
  for (u32 j = t; j < nseg; j += 256) {
    u32 lo = 0, hi = nr;  // first range with start > j
    while (lo < hi) {
      u32 mid = (lo + hi) >> 1;
      if (cov[2 * mid] <= j) lo = mid + 1;
      else hi = mid;
    }
    const bool covered = lo > 0 && j < cov[2 * (lo - 1) + 1];
    ws.active[c0 + j] = covered ? 0u : 1u;
    if (j == 0) ws.entry_idx[c0] = 0;
  }
  __syncthreads();
  for (u32 k = t; k + 1 < nseg; k += 256) {
    if (!ws.active[c0 + k]) continue;
    const u32 nx = ws.conv_chain[c0 + k];
    if (nx < nseg) ws.entry_idx[c0 + nx] = ws.conv_idx[c0 + k];
  }
  __syncthreads();

  // 5. output count of each chain; 6. offsets
  base = 0;
  for (u32 j0 = 0; j0 < nseg; j0 += 256) {
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
    if (j < nseg) ws.out_off[c0 + j] = base + pos;
    base += tot;
  }
  if (t == 0) *F.out_count = base;
}

// Compaction: one wave per chain of a multi-segment file copies its exact
// part; a continuation longer than its buffer is regenerated by walking on.
__global__ __launch_bounds__(256) void compact_kernel(const FileDesc* __restrict__ files, ChainWs ws,
                                                      const u32* __restrict__ chains, u32 nchains) {
  const u32 lane = lane_id();
  const u32 w = blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6);
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
    const u32 cc = ws.cont_cnt[chain];
    const u32 stored = cc < ws.cont_cap ? cc : ws.cont_cap;
    const u64* cont = ws.cont + ws.cont_off[chain];
    for (u32 i = 0; i < stored; i += 64) {
      const u32 ii = i + lane;
      if (ii < stored && o + (ii - i) < cap) out[o + (ii - i)] = cont[ii];
      o += (stored - i < 64) ? stored - i : 64;
    }
    if (cc > stored) {
      Chain ch;
      chain_init(ch, F);
      u64 x = cont[stored - 1];
      for (u32 i = stored; i < cc; i++) {
        x = next_cut(ch, x);
        if (lane == 0 && o < cap) out[o] = x;
        o++;
      }
    }
  }
  if (last || ws.conv_chain[chain] == F.nseg) {
    if (lane == 0 && o < cap) out[o] = F.n;
  }
}

// ---------------------------------------------------------------------------
// Launchers (host side)
// ---------------------------------------------------------------------------

hipError_t launch_mark(const FileDesc* d_files, u32 nfiles, u64 total_spans, u32 span_blocks, u32* d_counters,
                       hipStream_t st) {
  const u64 groups = (total_spans + kWavesPerGroup - 1) / kWavesPerGroup;
  dim3 grid((u32)(groups ? groups : 1)), block(256);
  switch (span_blocks) {
    case 4: hipLaunchKernelGGL(mark_kernel<4>, grid, block, 0, st, d_files, nfiles, total_spans, d_counters); break;
    case 16: hipLaunchKernelGGL(mark_kernel<16>, grid, block, 0, st, d_files, nfiles, total_spans, d_counters); break;
    default: hipLaunchKernelGGL(mark_kernel<8>, grid, block, 0, st, d_files, nfiles, total_spans, d_counters); break;
  }
  return hipGetLastError();
}

hipError_t launch_chains(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32 groups,
                         hipStream_t st) {
  if (!nitems) return hipSuccess;
  hipLaunchKernelGGL(chains_kernel, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems);
  return hipGetLastError();
}

hipError_t launch_continue(const FileDesc* d_files, const ChainWs& ws, const u32* d_order, u32 nitems, u32 groups,
                           hipStream_t st) {
  if (!nitems) return hipSuccess;
  hipLaunchKernelGGL(continue_kernel, dim3(groups), dim3(256), 0, st, d_files, ws, d_order, nitems);
  return hipGetLastError();
}

hipError_t launch_stitch(const FileDesc* d_files, const ChainWs& ws, const u32* d_multi, u32 nmulti, hipStream_t st) {
  if (!nmulti) return hipSuccess;
  hipLaunchKernelGGL(stitch_kernel, dim3(nmulti), dim3(256), 0, st, d_files, ws, d_multi, nmulti);
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
