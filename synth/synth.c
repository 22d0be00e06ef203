/*
 * Seeded synthetic workload generators.
 *
 * This module draws bytes, sizes and arrival times; it contains none of the
 * chunking arithmetic.  Both the CPU oracle's tests and the GPU path's tests
 * and benchmarks take their inputs from here, so the two sides see identical
 * bytes.  Every generator is counter based: value i of stream `tag` under
 * `seed` is a pure function of (seed, tag, i), so any slice can be produced
 * independently and in parallel.
 *
 * The workloads stand in for the paper's backup / VM-image / snapshot data
 * sets (Table II), which are not available: uniform random bytes, a mixed
 * "backup-like" stream (incompressible, text-like and low-entropy blocks), a
 * snapshot series built by seeded edits, log-normal file sizes and Poisson
 * request arrivals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

/* splitmix64 finaliser (Steele, Lea, Flood 2014). */
static inline uint64_t mix64(uint64_t z) {
  z += GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of one named random stream under a seed. */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
  return mix64(mix64(seed) ^ (tag * 0xD1B54A32D192ED03ULL));
}

/* Value i of a keyed stream. */
static inline uint64_t draw(uint64_t key, uint64_t i) {
  return mix64(key ^ (i * GOLDEN));
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double draw_unit(uint64_t key, uint64_t i) {
  return (double)(draw(key, i) >> 11) * (1.0 / 9007199254740992.0);
}

enum {
  TAG_UNIFORM = 1,
  TAG_BLOCK_KIND = 2,
  TAG_TEXT = 3,
  TAG_TEXT_PERM = 4,
  TAG_LOWENT = 5,
  TAG_EDIT = 6,
  TAG_EDIT_BYTES = 7,
  TAG_SIZES = 8,
  TAG_ARRIVAL = 9,
  TAG_MISC = 10,
};

uint64_t synth_draw(uint64_t seed, uint64_t tag, uint64_t i) {
  return draw(stream_key(seed, tag), i);
}

/* ------------------------------------------------------------------ */
/* Uniform bytes: byte i is byte (i mod 8) of draw(key, i / 8).        */
/* ------------------------------------------------------------------ */
static void uniform_fill(uint64_t key, uint64_t offset, uint64_t n, uint8_t *out) {
  uint64_t i = 0;
  while (i < n && ((offset + i) & 7)) {
    uint64_t g = offset + i;
    out[i] = (uint8_t)(draw(key, g >> 3) >> ((g & 7) * 8));
    i++;
  }
  for (; i + 8 <= n; i += 8) {
    uint64_t v = draw(key, (offset + i) >> 3);
    memcpy(out + i, &v, 8); /* little-endian host */
  }
  for (; i < n; i++) {
    uint64_t g = offset + i;
    out[i] = (uint8_t)(draw(key, g >> 3) >> ((g & 7) * 8));
  }
}

void synth_uniform(uint64_t seed, uint64_t offset, uint64_t n, uint8_t *out) {
  uint64_t key = stream_key(seed, TAG_UNIFORM);
  const uint64_t chunk = 1ULL << 20;
  int64_t nchunks = (int64_t)((n + chunk - 1) / chunk);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; c++) {
    uint64_t lo = (uint64_t)c * chunk;
    uint64_t len = n - lo < chunk ? n - lo : chunk;
    uniform_fill(key, offset + lo, len, out + lo);
  }
}

/* ------------------------------------------------------------------ */
/* Mixed "backup-like" content in 1 MiB blocks.                        */
/*   block kind = draw(kind_key, block) mod 100:                       */
/*     [0, 50)  uniform random bytes                                   */
/*     [50, 80) text-like: Zipf(s = 1.1) over 64 printable symbols     */
/*     [80,100) low-entropy: runs of length U[256, 65536], each all    */
/*              zero or a repeated random 16-byte pattern              */
/* The Zipf sampler is an inverse-CDF lookup on a 16-bit uniform; the  */
/* rank -> symbol map is a seeded permutation of 0x20..0x5F.           */
/* ------------------------------------------------------------------ */
#define MIX_BLOCK (1ULL << 20)

typedef struct {
  uint8_t table[65536];
} zipf_table;

static void build_zipf(uint64_t seed, double s, zipf_table *zt) {
  uint8_t sym[64];
  for (int i = 0; i < 64; i++) sym[i] = (uint8_t)(0x20 + i);
  uint64_t pk = stream_key(seed, TAG_TEXT_PERM);
  for (int i = 63; i > 0; i--) { /* Fisher-Yates */
    int j = (int)(draw(pk, (uint64_t)i) % (uint64_t)(i + 1));
    uint8_t t = sym[i];
    sym[i] = sym[j];
    sym[j] = t;
  }
  double w[64], tot = 0.0;
  for (int r = 0; r < 64; r++) {
    w[r] = 1.0 / pow((double)(r + 1), s);
    tot += w[r];
  }
  double cdf = 0.0;
  int r = 0;
  for (int u = 0; u < 65536; u++) {
    double x = ((double)u + 0.5) / 65536.0;
    while (r < 63 && x >= (cdf + w[r] / tot)) {
      cdf += w[r] / tot;
      r++;
    }
    zt->table[u] = sym[r];
  }
}

int synth_block_kind(uint64_t seed, uint64_t block) {
  uint64_t v = draw(stream_key(seed, TAG_BLOCK_KIND), block) % 100;
  return v < 50 ? 0 : (v < 80 ? 1 : 2);
}

static void mixed_block(uint64_t seed, uint64_t block, const zipf_table *zt, uint8_t *blk) {
  int kind = synth_block_kind(seed, block);
  uint64_t base = block * MIX_BLOCK;
  if (kind == 0) {
    uniform_fill(stream_key(seed, TAG_UNIFORM), base, MIX_BLOCK, blk);
  } else if (kind == 1) {
    uint64_t tk = stream_key(seed, TAG_TEXT);
    for (uint64_t i = 0; i < MIX_BLOCK; i += 4) {
      uint64_t v = draw(tk, (base + i) >> 2);
      blk[i + 0] = zt->table[(v >> 0) & 0xFFFF];
      blk[i + 1] = zt->table[(v >> 16) & 0xFFFF];
      blk[i + 2] = zt->table[(v >> 32) & 0xFFFF];
      blk[i + 3] = zt->table[(v >> 48) & 0xFFFF];
    }
  } else {
    uint64_t lk = stream_key(seed, TAG_LOWENT ^ (block << 8));
    uint64_t pos = 0, ctr = 0;
    while (pos < MIX_BLOCK) {
      uint64_t len = 256 + draw(lk, ctr++) % (65536 - 256 + 1);
      if (len > MIX_BLOCK - pos) len = MIX_BLOCK - pos;
      uint64_t sel = draw(lk, ctr++);
      if (sel & 1) {
        uint8_t pat[16];
        uint64_t a = draw(lk, ctr++), b = draw(lk, ctr++);
        memcpy(pat, &a, 8);
        memcpy(pat + 8, &b, 8);
        for (uint64_t i = 0; i < len; i++) blk[pos + i] = pat[i & 15];
      } else {
        memset(blk + pos, 0, len);
      }
      pos += len;
    }
  }
}

/* Bytes [offset, offset + n) of the mixed stream under `seed`. */
void synth_mixed(uint64_t seed, uint64_t offset, uint64_t n, uint8_t *out) {
  if (n == 0) return;
  zipf_table *zt = (zipf_table *)malloc(sizeof(zipf_table));
  build_zipf(seed, 1.1, zt);
  uint64_t b0 = offset / MIX_BLOCK, b1 = (offset + n - 1) / MIX_BLOCK;
  int64_t nb = (int64_t)(b1 - b0 + 1);
#pragma omp parallel
  {
    uint8_t *blk = (uint8_t *)malloc(MIX_BLOCK);
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < nb; k++) {
      uint64_t block = b0 + (uint64_t)k;
      uint64_t lo = block * MIX_BLOCK, hi = lo + MIX_BLOCK;
      uint64_t a = lo > offset ? lo : offset;
      uint64_t e = hi < offset + n ? hi : offset + n;
      if (a == lo && e == hi) {
        mixed_block(seed, block, zt, out + (a - offset));
      } else {
        mixed_block(seed, block, zt, blk);
        memcpy(out + (a - offset), blk + (a - lo), e - a);
      }
    }
    free(blk);
  }
  free(zt);
}

/* ------------------------------------------------------------------ */
/* Snapshot series: version v+1 = version v after `nedits` edits.      */
/* Each edit: op uniform in {insert, delete, overwrite}, length        */
/* U[1, maxlen], position uniform over the offsets where it fits; new  */
/* bytes uniform.  Edits are applied in order to a piece table and the */
/* result is materialised once.                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  int src; /* 0 = previous version, 1 = fresh bytes */
  uint64_t off, len;
} piece;

static int pieces_split(piece *p, int np, uint64_t at) {
  /* ensure a piece boundary at logical offset `at`; returns new count */
  uint64_t pos = 0;
  for (int i = 0; i < np; i++) {
    if (at == pos) return np;
    if (at < pos + p[i].len) {
      memmove(p + i + 2, p + i + 1, (size_t)(np - i - 1) * sizeof(piece));
      uint64_t cut = at - pos;
      p[i + 1].src = p[i].src;
      p[i + 1].off = p[i].off + cut;
      p[i + 1].len = p[i].len - cut;
      p[i].len = cut;
      return np + 1;
    }
    pos += p[i].len;
  }
  return np;
}

static int piece_index_at(const piece *p, int np, uint64_t at) {
  uint64_t pos = 0;
  for (int i = 0; i < np; i++) {
    if (pos == at) return i;
    pos += p[i].len;
  }
  return np;
}

/* Returns the size of the new version, or 0 if `out` is too small.
 * `fresh` must hold at least nedits * maxlen bytes of scratch. */
uint64_t synth_snapshot_next(const uint8_t *prev, uint64_t prev_size, uint64_t seed, uint64_t version,
                             uint64_t nedits, uint64_t maxlen, uint8_t *fresh, uint8_t *out, uint64_t out_cap) {
  int cap = (int)(3 * nedits + 4);
  piece *p = (piece *)malloc((size_t)cap * sizeof(piece));
  int np = 1;
  p[0].src = 0;
  p[0].off = 0;
  p[0].len = prev_size;
  uint64_t size = prev_size, fresh_used = 0;
  uint64_t ek = stream_key(seed ^ (version * 0x100000001B3ULL), TAG_EDIT);
  uint64_t bk = stream_key(seed ^ (version * 0x100000001B3ULL), TAG_EDIT_BYTES);
  uint64_t ctr = 0;
  for (uint64_t e = 0; e < nedits; e++) {
    int op = (int)(draw(ek, ctr++) % 3);
    uint64_t len = 1 + draw(ek, ctr++) % maxlen;
    uint64_t r = draw(ek, ctr++);
    if (op != 0 && len > size) op = 0; /* nothing to delete/overwrite: insert */
    if (op == 0) {                     /* insert `len` fresh bytes at pos in [0, size] */
      uint64_t pos = r % (size + 1);
      np = pieces_split(p, np, pos);
      int i = piece_index_at(p, np, pos);
      memmove(p + i + 1, p + i, (size_t)(np - i) * sizeof(piece));
      p[i].src = 1;
      p[i].off = fresh_used;
      p[i].len = len;
      np++;
      uniform_fill(bk, fresh_used, len, fresh + fresh_used);
      fresh_used += len;
      size += len;
    } else { /* delete or overwrite [pos, pos+len), pos in [0, size-len] */
      uint64_t pos = r % (size - len + 1);
      np = pieces_split(p, np, pos);
      np = pieces_split(p, np, pos + len);
      int i = piece_index_at(p, np, pos), j = piece_index_at(p, np, pos + len);
      memmove(p + i, p + j, (size_t)(np - j) * sizeof(piece));
      np -= (j - i);
      if (op == 1) {
        size -= len;
      } else {
        memmove(p + i + 1, p + i, (size_t)(np - i) * sizeof(piece));
        p[i].src = 1;
        p[i].off = fresh_used;
        p[i].len = len;
        np++;
        uniform_fill(bk, fresh_used, len, fresh + fresh_used);
        fresh_used += len;
      }
    }
  }
  if (size > out_cap) {
    free(p);
    return 0;
  }
  uint64_t pos = 0;
  for (int i = 0; i < np; i++) {
    memcpy(out + pos, (p[i].src ? fresh : prev) + p[i].off, p[i].len);
    pos += p[i].len;
  }
  free(p);
  return size;
}

/* ------------------------------------------------------------------ */
/* Sizes and arrivals.                                                 */
/* ------------------------------------------------------------------ */
/* Standard normal via Box-Muller on two counter draws. */
static double normal01(uint64_t key, uint64_t i) {
  double u1 = draw_unit(key, 2 * i), u2 = draw_unit(key, 2 * i + 1);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* clamp(round(exp(ln(median) + sigma * N(0,1))), lo, hi) */
void synth_lognormal_sizes(uint64_t seed, uint64_t count, double median, double sigma, uint64_t lo, uint64_t hi,
                           uint64_t *out) {
  uint64_t key = stream_key(seed, TAG_SIZES);
  for (uint64_t i = 0; i < count; i++) {
    double v = exp(log(median) + sigma * normal01(key, i));
    double r = floor(v + 0.5);
    uint64_t s = r < (double)lo ? lo : (r > (double)hi ? hi : (uint64_t)r);
    out[i] = s;
  }
}

/* Poisson process: cumulative exponential inter-arrival times (seconds). */
void synth_poisson_arrivals(uint64_t seed, uint64_t count, double rate, double *out) {
  uint64_t key = stream_key(seed, TAG_ARRIVAL);
  double t = 0.0;
  for (uint64_t i = 0; i < count; i++) {
    double u = draw_unit(key, i);
    t += -log(1.0 - u) / rate;
    out[i] = t;
  }
}

/* Uniform integers in [0, bound) (bound >= 1), e.g. slice offsets. */
void synth_uniform_ints(uint64_t seed, uint64_t tag, uint64_t count, uint64_t bound, uint64_t *out) {
  uint64_t key = stream_key(seed, TAG_MISC ^ (tag << 8));
  for (uint64_t i = 0; i < count; i++) out[i] = draw(key, i) % bound;
}
