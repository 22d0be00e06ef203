// Exact-content deduplication statistics (space savings, Eq. 1 of the paper)
// over chunk lists produced by the library.
#include <cstring>
#include <unordered_map>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

namespace {

struct Key {
  u64 a, b;
  bool operator==(const Key& o) const { return a == o.a && b == o.b; }
};
struct KeyHash {
  size_t operator()(const Key& k) const { return (size_t)(k.a ^ (k.b * 0x9E3779B97F4A7C15ull)); }
};

inline u64 mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Two independent 64-bit lanes over 8-byte words (tail zero-padded) plus length.
Key hash128(const uint8_t* p, u64 len) {
  u64 h1 = 0x243F6A8885A308D3ull ^ len, h2 = 0x13198A2E03707344ull ^ (len * 0x9E3779B97F4A7C15ull);
  u64 i = 0;
  for (; i + 8 <= len; i += 8) {
    u64 w;
    memcpy(&w, p + i, 8);
    h1 = mix(h1 ^ w) + 0x9E3779B97F4A7C15ull;
    h2 = mix(h2 + w * 0xD1B54A32D192ED03ull) ^ (h2 >> 17);
  }
  if (i < len) {
    u64 w = 0;
    memcpy(&w, p + i, len - i);
    h1 = mix(h1 ^ w ^ 0xA5);
    h2 = mix(h2 + w * 0xD1B54A32D192ED03ull + 0x5A);
  }
  return Key{mix(h1 ^ (h2 << 1)), mix(h2 + h1)};
}

struct Ref {
  u32 buf;
  u64 start, len;
};

}  // namespace

}  // namespace seqcdc

using namespace seqcdc;

extern "C" int seqcdc_dedup_stats(const uint8_t* const* bufs, const uint64_t* const* cuts, const uint64_t* counts,
                                  uint32_t nbuf, uint64_t* orig_bytes, uint64_t* unique_bytes, double* savings,
                                  double* ratio) {
  if (nbuf && (!bufs || !cuts || !counts)) return fail(SEQCDC_EINVAL, "NULL argument");
  std::unordered_map<Key, std::vector<Ref>, KeyHash> seen;
  u64 orig = 0, uniq = 0;
  for (u32 b = 0; b < nbuf; b++) {
    u64 start = 0;
    for (u64 i = 0; i < counts[b]; i++) {
      const u64 end = cuts[b][i];
      if (end < start) return fail(SEQCDC_EINVAL, "buffer %u: cuts must increase", b);
      const u64 len = end - start;
      const uint8_t* p = bufs[b] + start;
      Key k = hash128(p, len);
      auto& refs = seen[k];
      bool dup = false;
      for (const Ref& r : refs)
        if (r.len == len && memcmp(bufs[r.buf] + r.start, p, len) == 0) {
          dup = true;
          break;
        }
      if (!dup) {
        refs.push_back(Ref{b, start, len});
        uniq += len;
      }
      orig += len;
      start = end;
    }
  }
  if (orig_bytes) *orig_bytes = orig;
  if (unique_bytes) *unique_bytes = uniq;
  if (savings) *savings = orig ? (double)(orig - uniq) / (double)orig : 0.0;
  if (ratio) *ratio = uniq ? (double)orig / (double)uniq : 1.0;
  return SEQCDC_OK;
}
