// Deduplication on the device, the stage after chunking (Sec. II): every
// chunk gets a SHA-256 fingerprint, fingerprints go into an open-addressing
// table, and a chunk whose fingerprint is already there is compared byte for
// byte with the chunk that holds the entry.  The space savings of Eq. 1 follow
// from the bytes of the chunks that are not duplicates.
//
// SHA-256 is FIPS 180-4: 512-bit blocks, the message padded with a 1 bit,
// zeros and its 64-bit bit length, eight 32-bit working variables, 64 rounds
// per block.  One thread hashes one chunk (the blocks of a message are
// sequential); a chunk's bytes are read as aligned 32-bit words realigned to
// its first byte, so any chunk start works.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_device.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

// FIPS 180-4 Sec. 4.2.2: the first 32 bits of the fractional parts of the
// cube roots of the first 64 primes.
__constant__ u32 kSha256K[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u,
    0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u,
    0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
    0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u,
    0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u,
    0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
    0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
    0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};

// FIPS 180-4 Sec. 5.3.3: the first 32 bits of the fractional parts of the
// square roots of the first 8 primes.
constexpr u32 kSha256H0[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                              0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

__device__ __forceinline__ u32 rotr(u32 x, u32 n) { return __builtin_amdgcn_alignbit(x, x, n); }

// Three-input bitwise functions as one v_bitop3 each: bit i of the 8-bit table
// is the result for the input bits (x, y, z) = (i >> 2, (i >> 1) & 1, i & 1).
__device__ __forceinline__ u32 xor3(u32 x, u32 y, u32 z) { return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96); }
__device__ __forceinline__ u32 choose(u32 x, u32 y, u32 z) { return __builtin_amdgcn_bitop3_b32(x, y, z, 0xCA); }
__device__ __forceinline__ u32 majority(u32 x, u32 y, u32 z) { return __builtin_amdgcn_bitop3_b32(x, y, z, 0xE8); }
__device__ __forceinline__ u32 bswap32(u32 x) { return __builtin_amdgcn_perm(0u, x, 0x00010203u); }

// One 64-byte block into the state (FIPS 180-4 Sec. 6.2.2), the message
// schedule kept as a rolling window of 16 words.
__device__ __forceinline__ void sha256_block(u32 st[8], u32 w[16]) {
  u32 a = st[0], b = st[1], c = st[2], d = st[3], e = st[4], f = st[5], g = st[6], h = st[7];
#pragma unroll
  for (int i = 0; i < 64; i++) {
    u32 wi;
    if (i < 16) {
      wi = w[i];
    } else {
      const u32 w15 = w[(i - 15) & 15], w2 = w[(i - 2) & 15];
      const u32 s0 = xor3(rotr(w15, 7), rotr(w15, 18), w15 >> 3);  // sigma0 (Sec. 4.1.2)
      const u32 s1 = xor3(rotr(w2, 17), rotr(w2, 19), w2 >> 10);   // sigma1
      wi = w[i & 15] + s0 + w[(i - 7) & 15] + s1;
      w[i & 15] = wi;
    }
    const u32 S1 = xor3(rotr(e, 6), rotr(e, 11), rotr(e, 25));  // Sigma1 (Sec. 4.1.2)
    const u32 ch = choose(e, f, g);                              // Ch: f where e is 1, g where e is 0
    const u32 t1 = h + S1 + ch + kSha256K[i] + wi;
    const u32 S0 = xor3(rotr(a, 2), rotr(a, 13), rotr(a, 22));  // Sigma0
    const u32 maj = majority(a, b, c);                           // Maj
    const u32 t2 = S0 + maj;
    h = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + t2;
  }
  st[0] += a;
  st[1] += b;
  st[2] += c;
  st[3] += d;
  st[4] += e;
  st[5] += f;
  st[6] += g;
  st[7] += h;
}

// The 17 aligned 32-bit words from the one at or below p (they cover the 64
// bytes at p wherever p falls in a word).  Only words that hold a byte below
// `end` are read from there (such a word never crosses a page end); the
// others read the word at `safe`, a valid address: all their bytes lie at or
// past `end`, where words_from_raw ignores them.  Every word is one load in
// every lane, with no branch around it, so the loads of a block can be waited
// for as one group.
__device__ __forceinline__ void load_raw(const uint8_t* p, const uint8_t* end, const u32* safe, u32 d[17]) {
  const uintptr_t a = (uintptr_t)p;
  const u32 sh = (u32)(a & 3);
  const uintptr_t e = (uintptr_t)end;
#pragma unroll
  for (int j = 0; j < 17; j++) {
    const uintptr_t wa = a - sh + 4 * j;
    d[j] = *as_global(wa < e ? (const u32*)wa : safe);
  }
}

// The 16 big-endian message words of the 64 bytes at p (p + 64 <= end), or
// of the last part of a message: the bytes [p, end) followed, when `pad`, by
// the 0x80 byte at end - p (< 64) and zeros; all zeros when p > end.  d holds
// the words load_raw(p, end) read; their bytes at or past `end` are ignored.
__device__ __forceinline__ void words_from_raw(const u32 d[17], const uint8_t* p, const uint8_t* end, bool pad,
                                               u32 w[16]) {
  const uintptr_t a = (uintptr_t)p;
  const u32 sh = (u32)(a & 3);
  const uintptr_t e = (uintptr_t)end;
  // message bytes from p: none when p is past the end (the aligned word read
  // first may still hold the message's last bytes; they are masked off)
  const bool inside = a <= e;
  const uintptr_t left = inside ? e - a : 0;
  const u32 valid = left < 64 ? (u32)left : 64u;
  const bool pad_here = pad && inside && left < 64;  // the 0x80 byte falls in this block
#pragma unroll
  for (int k = 0; k < 16; k++) {
    u32 x = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);  // bytes 4k .. 4k+3 from p, little-endian
    const u32 o = 4 * k;
    if (o + 4 > valid) {  // the word holds the end of the message
      const u32 keep = valid > o ? valid - o : 0;  // 0..3 message bytes
      x = keep ? x & ((1u << (8 * keep)) - 1u) : 0u;
      if (pad_here && valid >= o && valid < o + 4) x |= 0x80u << (8 * (valid - o));
    }
    w[k] = bswap32(x);
  }
}

// The 16 bytes from byte sh (0..15) of the 32 bytes lo:hi (little-endian).
__device__ __forceinline__ void realign16(const uint4& lo, const uint4& hi, u32 sh, u32 out[4]) {
  const u32 w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  const u32 ws = sh >> 2, bs = sh & 3;
  u32 t[5];
#pragma unroll
  for (int k = 0; k < 5; k++) t[k] = ws == 0 ? w[k] : ws == 1 ? w[k + 1] : ws == 2 ? w[k + 2] : w[k + 3];
#pragma unroll
  for (int k = 0; k < 4; k++) out[k] = __builtin_amdgcn_alignbyte(t[k + 1], t[k], bs);
}

// The two aligned 16-byte vectors that hold the 16 bytes of the chunk
// [p, p + n) at off .. off + 15 (off < n; a multiple of 16), where sh = p mod
// 16: the vector holding p + off, and the next one only while it holds a byte
// of the chunk (an aligned vector never crosses a page end; otherwise the
// first is read twice).  realign16(lo, hi, sh) gives the 16 bytes (those at or
// past n unspecified).
__device__ __forceinline__ void chunk16_raw(const uint8_t* p, u64 n, u64 off, u32 sh, uint4& lo, uint4& hi) {
  const uintptr_t al = (uintptr_t)(p + off) - sh;
  const uintptr_t end = (uintptr_t)(p + n);
  lo = load16((const void*)al);
  hi = load16((const void*)(al + 16 < end ? al + 16 : al));
}

// A file of the call: its bytes, the range of its cut slots, its count.
struct DedupFile {
  const uint8_t* data;
  u64 slot0;               // first slot (index into d_cuts / digests)
  const u64* count;        // device: number of cuts
};

__device__ __forceinline__ u32 file_of_slot(const DedupFile* __restrict__ files, u32 nfiles, u64 slot) {
  u32 lo = 0, hi = nfiles;  // last file with slot0 <= slot
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (files[mid].slot0 <= slot) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Chunk `slot`: its file's bytes and [start, end); false for a slot past the file's count.
__device__ __forceinline__ bool chunk_of(const DedupFile* __restrict__ files, u32 nfiles, const u64* __restrict__ cuts,
                                         u64 slot, const uint8_t*& data, u64& start, u64& end) {
  const DedupFile& F = files[file_of_slot(files, nfiles, slot)];
  const u64 j = slot - F.slot0;
  if (j >= *F.count) return false;
  data = F.data;
  start = j ? cuts[slot - 1] : 0;
  end = cuts[slot];
  return true;
}

// Block b of the padded message of the len bytes at p (FIPS 180-4 Sec.
// 5.1.1) from the words load_raw(p + 64 b, p + len) read: the message bytes,
// the 0x80 byte right after them, zeros, and the 64-bit bit length in the last
// 8 bytes of the last of the nb blocks.  The same code serves every block
// (nothing at or past the end was read, and the 0x80 byte goes where the
// message ends inside the block).
__device__ __forceinline__ void padded_block(const u32 d[17], const uint8_t* p, u64 len, u64 b, u64 nb, u32 w[16]) {
  words_from_raw(d, p + 64 * b, p + len, true, w);
  if (b + 1 == nb) {
    w[14] = (u32)((len * 8) >> 32);
    w[15] = (u32)(len * 8);
  }
}

// Pass 1 with balanced lanes: each lane hashes chunk after chunk, and every
// step hashes one block of each lane's current message, so the lanes of a
// wave stay busy however the chunk lengths of neighbouring slots differ.  A
// wave takes slots from the global queue kBatch at a time (every lane
// executes that atomic, lane 0 adding kBatch, in wave-uniform control flow)
// and hands them in lane order (ranks by mbcnt) to the lanes that need a
// message after the current step: idle lanes, and lanes hashing the last
// block of theirs.  The words of the block a lane hashes at the next step (its
// message's next block, or the first block of the message it takes up next)
// are loaded during the current step, so the loads run while the current
// block's 64 rounds do.  A lane that was idle hashes an empty block for one
// step while its first block loads.  Slots past a file's count get a zero
// digest.  A wave ends once the queue is empty and its lanes have finished:
// every step either hashes a block or takes slots.
constexpr u32 kShaBatch = 64;

__global__ __launch_bounds__(256) void sha_queue_kernel(const DedupFile* __restrict__ files, u32 nfiles,
                                                        const u64* __restrict__ cuts, u64 nslots, u32* digests,
                                                        unsigned long long* next) {
  const u32* safe = (const u32*)cuts;  // a valid word for the loads that read nothing
  u64 wb = 0, we = 0;      // wave-uniform: the wave's batch of slots [wb, we)
  bool exhausted = false;  // wave-uniform: the queue had no slot left
  // the lane's current message: block b of nb is hashed at the next step
  u64 slot = 0;
  const uint8_t* p = nullptr;
  u64 len = 0, b = 0, nb = 1;
  bool busy = false;
  // the message the lane takes up after the current one
  u64 nslot = 0;
  const uint8_t* np = nullptr;
  u64 nlen = 0;
  bool has_next = false;
  u32 st[8];
#pragma unroll
  for (int i = 0; i < 8; i++) st[i] = 0;
  u32 dc[17];  // the words of block b, loaded during the previous step
#pragma unroll
  for (int j = 0; j < 17; j++) dc[j] = 0;
  for (;;) {
    const bool want = !has_next && (!busy || b + 1 == nb);
    const u64 need = ballot(want);
    if (need && !exhausted) {
      if (wb == we) {
        const unsigned long long v = atomicAdd(next, lane_id() == 0 ? (unsigned long long)kShaBatch : 0ull);
        wb = readlane64((u64)v, 0);
        we = wb + kShaBatch;
        if (wb >= nslots) exhausted = true;
      }
      if (!exhausted) {
        const u64 avail = we - wb;
        const u32 rank = __builtin_amdgcn_mbcnt_hi((u32)(need >> 32), __builtin_amdgcn_mbcnt_lo((u32)need, 0u));
        if (want && rank < avail) {
          const u64 sl = wb + rank;
          if (sl < nslots) {
            const uint8_t* data;
            u64 start, end;
            if (chunk_of(files, nfiles, cuts, sl, data, start, end)) {
              nslot = sl;
              np = data + start;
              nlen = end - start;
              has_next = true;
            } else {  // past its file's count
              uint4* dst = (uint4*)(digests + 8 * sl);
              dst[0] = make_uint4(0, 0, 0, 0);
              dst[1] = make_uint4(0, 0, 0, 0);
            }
          }
        }
        const u64 k = (u64)__popcll(need);
        wb += k < avail ? k : avail;
      }
    }
    if (!ballot(busy || has_next)) {
      if (exhausted) break;  // no slot left and no lane with a message
      continue;              // the slots taken were past their files' counts: take more
    }
    // the words of the block hashed at the next step, loaded while this one is hashed
    u32 dn[17];
    {
      const bool more = busy && b + 1 < nb;
      const uint8_t* q = more ? p + 64 * (b + 1) : has_next ? np : nullptr;
      const uint8_t* qe = more ? p + len : has_next ? np + nlen : nullptr;
      load_raw(q, qe, safe, dn);
    }
    // one block of every busy lane's message; the other lanes hash an empty message
    u32 w[16];
    padded_block(dc, busy ? p : nullptr, busy ? len : 0, busy ? b : 0, busy ? nb : 1, w);
    u32 s2[8];
#pragma unroll
    for (int i = 0; i < 8; i++) s2[i] = st[i];
    sha256_block(s2, w);
#pragma unroll
    for (int j = 0; j < 17; j++) dc[j] = dn[j];
    // the loads complete here: after the rounds (s2[0] depends on all of
    // them), before the digest stores below (a wait placed after those stores
    // would wait for them too: one counter covers loads and stores)
    asm volatile("" : "+v"(dc[0]), "+v"(dc[1]), "+v"(dc[2]), "+v"(dc[3]), "+v"(dc[4]), "+v"(dc[5]), "+v"(dc[6]),
                 "+v"(dc[7]), "+v"(dc[8]), "+v"(s2[0]) : : "memory");
    asm volatile("" : "+v"(dc[9]), "+v"(dc[10]), "+v"(dc[11]), "+v"(dc[12]), "+v"(dc[13]), "+v"(dc[14]),
                 "+v"(dc[15]), "+v"(dc[16]) : : "memory");
    if (busy) {
#pragma unroll
      for (int i = 0; i < 8; i++) st[i] = s2[i];
      b++;
      if (b == nb) {
        uint4* dst = (uint4*)(digests + 8 * slot);
        dst[0] = make_uint4(st[0], st[1], st[2], st[3]);
        dst[1] = make_uint4(st[4], st[5], st[6], st[7]);
        busy = false;
      }
    }
    if (!busy && has_next) {  // take up the next message: its first block is in dc
      slot = nslot;
      p = np;
      len = nlen;
      b = 0;
      nb = (len + 8) / 64 + 1;
      busy = true;
      has_next = false;
#pragma unroll
      for (int i = 0; i < 8; i++) st[i] = kSha256H0[i];
    }
  }
}

constexpr u32 kNoOwner = 0xFFFFFFFFu;

// Pass 2: every chunk enters the table of 2^k 64-bit entries (tag: the
// digest's first word; value: slot + 1), probing linearly from its second
// word.  A chunk that finds an entry with its full digest records that
// entry's slot as its owner; the others own their entry.
__global__ __launch_bounds__(256) void insert_kernel(const DedupFile* __restrict__ files, u32 nfiles,
                                                     const u64* __restrict__ cuts, u64 nslots,
                                                     const u32* __restrict__ digests, u64* table, u64 mask,
                                                     u32* owner) {
  const u64 slot = (u64)blockIdx.x * 256 + threadIdx.x;
  if (slot >= nslots) return;
  const uint8_t* data;
  u64 start, end;
  if (!chunk_of(files, nfiles, cuts, slot, data, start, end)) {
    owner[slot] = kNoOwner;
    return;
  }
  const u32* h = digests + 8 * slot;
  const u64 entry = ((u64)h[0] << 32) | (u64)(slot + 1);
  u64 pos = h[1] & mask;
  for (u64 probe = 0; probe <= mask; probe++, pos = (pos + 1) & mask) {
    const u64 prev = atomicCAS((unsigned long long*)&table[pos], 0ull, (unsigned long long)entry);
    if (prev == 0) {  // the entry is this chunk's
      owner[slot] = kNoOwner;
      return;
    }
    if ((u32)(prev >> 32) != h[0]) continue;
    const u64 other = (prev & 0xFFFFFFFFull) - 1;
    const u32* g = digests + 8 * other;
    bool same = true;
#pragma unroll
    for (int i = 1; i < 8; i++) same = same && g[i] == h[i];
    if (same) {
      owner[slot] = (u32)other;
      return;
    }
  }
  owner[slot] = kNoOwner;  // unreachable: the table has more entries than chunks
}

// Pass 3: one wave per 64 slots.  Each lane looks up its slot's chunk and
// the chunk that owns its fingerprint (so the dependent lookups of 64 slots
// run together); a chunk with no owner is unique, and a chunk whose owner has
// another length is unique.  The wave then compares each remaining candidate
// with its owner byte for byte, 4 KiB at a time (each lane 4 x 16 bytes of
// both, read as aligned 16-byte vectors and realigned, all loads in flight
// together): a candidate is a duplicate only if all bytes are equal.  The bytes of the unique chunks and of all chunks are
// summed over the wave, then into the totals.
__global__ __launch_bounds__(256) void verify_kernel(const DedupFile* __restrict__ files, u32 nfiles,
                                                     const u64* __restrict__ cuts, u64 nslots,
                                                     const u32* __restrict__ owner, u64* totals) {
  const u32 lane = lane_id();
  const u64 slot = ((u64)blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6)) * 64 + lane;
  u64 orig = 0, uniq = 0, len = 0;
  const uint8_t* pa = nullptr;
  const uint8_t* pb = nullptr;
  bool cand = false;
  const uint8_t* data;
  u64 start, end;
  if (slot < nslots && chunk_of(files, nfiles, cuts, slot, data, start, end)) {
    len = end - start;
    orig = len;
    uniq = len;
    pa = data + start;
    const u32 o = owner[slot];
    if (o != kNoOwner) {
      const uint8_t* odata;
      u64 ostart, oend;
      chunk_of(files, nfiles, cuts, o, odata, ostart, oend);
      cand = oend - ostart == len;
      pb = odata + ostart;
    }
  }
  // the candidates, one after another over the whole wave
  for (u64 m = ballot(cand); m; m &= m - 1) {
    const u32 l = ctz64(m);
    const u64 n = readlane64(len, l);
    const uint8_t* a = (const uint8_t*)readlane64((u64)pa, l);
    const uint8_t* b = (const uint8_t*)readlane64((u64)pb, l);
    const u32 sha = (u32)((uintptr_t)a & 15), shb = (u32)((uintptr_t)b & 15);
    bool same = true;
    for (u64 base = 0; same && base < n; base += 4096) {
      uint4 alo[4], ahi[4], blo[4], bhi[4];
      u32 valid[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {  // every load first, then the compares
        const u64 off = base + 1024ull * u + 16ull * lane;
        const bool in = off < n;
        const u64 oc = in ? off : 0;  // lanes past the end read the chunk's first bytes and compare none
        valid[u] = in ? (n - off < 16 ? (u32)(n - off) : 16u) : 0u;
        chunk16_raw(a, n, oc, sha, alo[u], ahi[u]);
        chunk16_raw(b, n, oc, shb, blo[u], bhi[u]);
      }
      u32 diff = 0;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        u32 va[4], vb[4];
        realign16(alo[u], ahi[u], sha, va);
        realign16(blo[u], bhi[u], shb, vb);
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const u32 v = valid[u] > 4u * k ? valid[u] - 4u * k : 0u;  // bytes of word k that belong to the chunk
          const u32 mask = v >= 4 ? ~0u : (1u << (8 * v)) - 1u;
          diff |= (va[k] ^ vb[k]) & mask;
        }
      }
      same = ballot(diff != 0) == 0;
    }
    if (same && lane == l) uniq = 0;
  }
  const u64 so = wave_incl_scan64(orig), su = wave_incl_scan64(uniq);  // lane 63 holds the wave's sums
  if (lane == 63) {
    if (so) atomicAdd((unsigned long long*)&totals[0], (unsigned long long)so);
    if (su) atomicAdd((unsigned long long*)&totals[1], (unsigned long long)su);
  }
}

__global__ __launch_bounds__(256) void zero64_kernel(u64* p, u64 count) {
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < count; i += (u64)gridDim.x * 256) p[i] = 0;
}

}  // namespace seqcdc

using namespace seqcdc;

extern "C" int seqcdc_dedup_batch(seqcdc_plan* plan, const seqcdc_file* h_files, uint32_t nfiles,
                                  const uint64_t* d_cuts, const uint64_t* h_cut_offsets, const uint64_t* d_counts,
                                  uint32_t* d_digests, uint64_t* h_orig, uint64_t* h_unique, void* stream) {
  if (!plan || !h_files || !h_cut_offsets || !d_counts || !h_orig || !h_unique)
    return fail(SEQCDC_EINVAL, "NULL argument");
  if (nfiles == 0) {
    *h_orig = *h_unique = 0;
    return SEQCDC_OK;
  }
  if (!d_cuts) return fail(SEQCDC_EINVAL, "NULL cut array");
  for (u32 f = 0; f < nfiles; f++) {
    if (h_cut_offsets[f + 1] < h_cut_offsets[f]) return fail(SEQCDC_EINVAL, "cut offsets must not decrease");
    if (h_files[f].n && !h_files[f].d_data) return fail(SEQCDC_EINVAL, "file %u: NULL data", f);
  }
  const u64 slot0 = h_cut_offsets[0];
  const u64 nslots = h_cut_offsets[nfiles] - slot0;
  if (nslots >= 0xFFFFFFFEull) return fail(SEQCDC_EINVAL, "too many cut slots");
  Plan* pl = (Plan*)plan;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> g(pl->mu);
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (pl->pending && pl->last_stream != st) {
    e = hipStreamWaitEvent(st, pl->call_done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  u64 cap = 1024;
  while (cap < 2 * nslots) cap <<= 1;
  int rc;
  std::vector<DedupFile> df(nfiles);
  for (u32 f = 0; f < nfiles; f++)
    df[f] = DedupFile{(const uint8_t*)h_files[f].d_data, h_cut_offsets[f] - slot0, d_counts + f};
  const size_t files_bytes = (nfiles * sizeof(DedupFile) + 255) & ~(size_t)255;
  const size_t dig_bytes = d_digests ? 0 : ((nslots * 32 + 255) & ~(size_t)255);
  const size_t owner_bytes = (nslots * 4 + 255) & ~(size_t)255;
  const size_t table_bytes = cap * 8;
  const size_t total = files_bytes + dig_bytes + owner_bytes + table_bytes + 256;
  if ((rc = pl->misc.reserve(total))) return rc;
  if ((rc = pl->readback.reserve(64))) return rc;
  char* base = (char*)pl->misc.p;
  DedupFile* d_files = (DedupFile*)base;
  u32* digests = d_digests ? d_digests : (u32*)(base + files_bytes);
  u32* owner = (u32*)(base + files_bytes + dig_bytes);
  u64* table = (u64*)(base + files_bytes + dig_bytes + owner_bytes);
  u64* totals = (u64*)(base + files_bytes + dig_bytes + owner_bytes + table_bytes);
  if ((rc = pl->staging.reserve(files_bytes))) return rc;
  if (pl->upload_pending) {
    e = hipEventSynchronize(pl->upload_done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    pl->upload_pending = false;
  }
  memcpy(pl->staging.p, df.data(), nfiles * sizeof(DedupFile));
  pl->uploaded_dev = nullptr;  // the table buffer no longer holds a chunking call's tables
  e = hipMemcpyAsync(d_files, pl->staging.p, nfiles * sizeof(DedupFile), hipMemcpyHostToDevice, st);
  const u64* cuts = d_cuts + slot0;
  const u32 grid = (u32)((nslots + 255) / 256);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(zero64_kernel, dim3(1024), dim3(256), 0, st, table, cap + 2);
    hipLaunchKernelGGL(zero64_kernel, dim3(1), dim3(256), 0, st, totals, (u64)3);  // orig, unique, SHA queue
    e = hipGetLastError();
  }
  if (e == hipSuccess && nslots) {
    // two waves per SIMD (fewer for small calls): each lane hashes enough
    // chunks that the ones still running when the queue empties are a small
    // part of the work (measured on a 2.5 GiB series: one or three waves per
    // SIMD were 10 % and 9 % slower)
    const u32 sha_groups = (u32)std::max<u64>(1, std::min<u64>((u64)pl->cus * 2, (nslots + 255) / 256));
    hipLaunchKernelGGL(sha_queue_kernel, dim3(sha_groups), dim3(256), 0, st, d_files, nfiles, cuts, nslots, digests,
                       (unsigned long long*)(totals + 2));
    hipLaunchKernelGGL(insert_kernel, dim3(grid), dim3(256), 0, st, d_files, nfiles, cuts, nslots,
                       (const u32*)digests, table, cap - 1, owner);
    hipLaunchKernelGGL(verify_kernel, dim3((u32)((nslots + 64 * kWavesPerGroup - 1) / (64 * kWavesPerGroup))), dim3(256),
                       0, st,
                       d_files, nfiles, cuts, nslots, (const u32*)owner, totals);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(pl->readback.p, totals, 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "seqcdc_dedup_batch");
  pl->pending = false;
  const u64* r = (const u64*)pl->readback.p;
  *h_orig = r[0];
  *h_unique = r[1];
  return SEQCDC_OK;
}
