// SeqCDC mark step on CDNA4 (gfx950): device functions of the mark kernel.
//
// The vector formulation of Sec. III-D, one wave per 1 KiB block: every byte
// pair becomes one favourable bit F and one opposing bit O; E, the AND of
// SeqLength-1 consecutive F bits, marks the bytes that end a candidate run
// (Sec. III-A).  The bits are written packed (EO16), plus one summary byte
// per 1 KiB block that says whether the block holds any run end.
#pragma once
#include <hip/hip_runtime.h>

#include "seqcdc_device.h"

namespace seqcdc {

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

// The raw loads of this lane for the 1 KiB block at file offset B: the
// aligned 16-byte chunk holding the lane's first byte and, for lane 63 of a
// stream that does not start on a 16-byte boundary, the chunk after it (the
// other lanes take theirs from their neighbour).  Both are issued before any
// is used, so a batch of blocks keeps all its loads in flight.  All loads are
// 16-byte aligned: such a chunk never straddles a page, so chunks that
// overlap the stream [data, data+n) are safe to read whole; bytes outside
// the stream are ignored by the caller.
struct BlockLoad {
  u32x4 lo, ext;
};

__device__ __forceinline__ void load_block(const uint8_t* data, u64 n, u64 B, BlockLoad& L) {
  const u32 lane = lane_id();
  const uintptr_t addr = (uintptr_t)data;
  const u32 r = (u32)(addr & 15);
  const u32x4* base = (const u32x4*)(addr - r);  // aligned view; byte q of the stream is at r + q
  const u64 first = (B >> 4) + lane;              // aligned chunk index of this lane
  const u64 end_chunk = (r + n + 15) >> 4;        // aligned chunks overlapping the stream
  L.lo = u32x4{0, 0, 0, 0};
  L.ext = u32x4{0, 0, 0, 0};
  if (first < end_chunk) L.lo = __builtin_nontemporal_load(as_global(base + first));
  if (r != 0 && lane == 63 && first + 1 < end_chunk) L.ext = __builtin_nontemporal_load(as_global(base + first + 1));
}

// The 16 stream bytes of this lane from its raw loads.
__device__ __forceinline__ void block_bytes(const uint8_t* data, const BlockLoad& L, u32 x[4]) {
  const u32 r = (u32)((uintptr_t)data & 15);
  if (r == 0) {
    x[0] = L.lo.x; x[1] = L.lo.y; x[2] = L.lo.z; x[3] = L.lo.w;
    return;
  }
  uint4 lo = make_uint4(L.lo.x, L.lo.y, L.lo.z, L.lo.w), hi;
  hi.x = __shfl_down(lo.x, 1);
  hi.y = __shfl_down(lo.y, 1);
  hi.z = __shfl_down(lo.z, 1);
  hi.w = __shfl_down(lo.w, 1);
  if (lane_id() == 63) hi = make_uint4(L.ext.x, L.ext.y, L.ext.z, L.ext.w);
  funnel16(lo, hi, r, x);
}

// 16 bytes at file offset B-16 (B >= 16) for the halo, wave-uniform.
__device__ __forceinline__ void load_halo(const uint8_t* data, u64 n, u64 B, u32 x[4]) {
  const uintptr_t addr = (uintptr_t)data;
  const u32 r = (u32)(addr & 15);
  const uint4* base = (const uint4*)(addr - r);
  const u64 c0 = (B - 16) >> 4;
  uint4 lo = load16(base + c0);
  if (r == 0) {
    x[0] = lo.x; x[1] = lo.y; x[2] = lo.z; x[3] = lo.w;
    return;
  }
  uint4 hi = load16(base + c0 + 1);  // overlaps byte B-1 < n, so it overlaps the stream
  funnel16(lo, hi, r, x);
}

// Marks the 1 KiB blocks [span * span_blocks, (span + 1) * span_blocks) of
// one file with one wave.  Blocks are loaded kMarkBatch at a time so that
// several loads are in flight per wave; the last byte and F bits of each block
// carry into the next through lane 63.
constexpr u32 kMarkBatch = 4;

__device__ __forceinline__ void mark_span(const FileDesc& F, u64 span, u32 span_blocks) {
  const u32 lane = lane_id();
  const uint8_t* data = F.data;
  const u64 n = F.n;
  const u32 down_is_fav = F.mode & 1;  // decreasing mode: favourable = byte below its predecessor
  // signed bytes: x ^ 0x80 orders as the signed value of x, so the unsigned compares then compare signed values
  const u32 flip = (F.mode & 2) ? 0x80808080u : 0u;
  const u32 runlen = F.sl - 1;
  SEQCDC_GLOBAL u32* __restrict__ eo = as_global(F.eo);
  SEQCDC_GLOBAL uint8_t* __restrict__ esum = as_global(F.esum);
  const u64 nblk = (n + kMarkBlock - 1) / kMarkBlock;
  u64 blk = span * span_blocks;
  const u64 blk_end = blk + span_blocks < nblk ? blk + span_blocks : nblk;

  u32 carry_byte = 0, carry_fav = 0;  // last byte / F bits of the 16 bytes before the block
  if (blk > 0 && blk < blk_end) {
    u32 h[4];
    load_halo(data, n, blk * kMarkBlock, h);
#pragma unroll
    for (int k = 0; k < 4; k++) h[k] ^= flip;
    u32 up, dn;
    compare16(h, 0u, up, dn);  // bit 0 is wrong (unknown predecessor) but is never used for SeqLength <= 16
    carry_fav = down_is_fav ? dn : up;
    carry_byte = h[3] >> 24;
  }

#pragma unroll 1
  for (; blk < blk_end; blk += kMarkBatch) {
    BlockLoad ld[kMarkBatch];
#pragma unroll
    for (u32 d = 0; d < kMarkBatch; d++) {
      if (blk + d < blk_end) load_block(data, n, (blk + d) * kMarkBlock, ld[d]);
    }
#pragma unroll
    for (u32 d = 0; d < kMarkBatch; d++) {
      if (blk + d >= blk_end) break;
      const u64 B = (blk + d) * kMarkBlock;
      u32 x[4];
      block_bytes(data, ld[d], x);
#pragma unroll
      for (int k = 0; k < 4; k++) x[k] ^= flip;
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
      const bool any_end = ballot(e != 0) != 0;  // run-end summary: one byte per 1 KiB block
      if (lane == 0) esum[blk + d] = any_end ? 1 : 0;
      carry_byte = readlane(last, 63);
      carry_fav = readlane(fav, 63);
    }
  }
}

// File of a global mark span: the last file whose first span is <= span.
// hint[i] is the file holding span 64 i (entries past the last span: the last
// file), so the search only covers the files that start among these 64 spans.
__device__ __forceinline__ u32 file_of_span(const FileDesc* __restrict__ files, const u32* __restrict__ hint,
                                            u64 span) {
  const u64 h = span / kHintSpans;
  u32 lo = hint[h], hi = hint[h + 1] + 1;
  while (hi - lo > 1) {
    u32 mid = (lo + hi) >> 1;
    if (files[mid].mark_span0 <= span) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace seqcdc
