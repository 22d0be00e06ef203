/*
 * SeqCDC CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded byte loop that states what SeqCDC computes,
 * written from the paper (Udayashankar & Al-Kiswany, "Vectorized
 * Sequence-Based Chunking for Data Deduplication", arXiv 2505.21194).  Only
 * the test-suite, the smoke check and the benchmark's CPU baseline may load
 * it.  It shares no code, header or table with the GPU library.
 *
 * Readings of the paper taken here (all listed in the design notes):
 *  - SeqLength counts BYTES in the monotone run (Sec. III-A; Sec. III-D uses
 *    SeqLength shifted registers and SeqLength-1 pairwise masks, and its
 *    worked example cuts after the three bytes 12 13 14 with SeqLength 3).
 *  - Monotone means strict; bytes are unsigned (Sec. III-D compares with
 *    cmpgt / cmplt).  An equal pair ends a run and is not opposing.
 *  - The boundary is the exclusive offset just past the last byte of the run
 *    (Sec. III-A "inserted at its end"; Sec. III-D "SeqLength bytes ahead of
 *    the first set bit").
 *  - Scanning of a chunk starts min - SeqLength bytes after its start, so the
 *    first candidate run may begin there (Sec. III-B).
 *  - The opposing-pair count is a running total since the chunk start or
 *    the last skip; a skip fires when it reaches SkipTrigger, at the later
 *    byte of the pair; the next SkipSize bytes are ignored and scanning
 *    resumes with fresh counters (Sec. III-C, Fig. 2 prose).
 *  - With no boundary, the chunk ends at start + max, or at the end of the
 *    stream (Sec. IV "Maximum chunk size"); a skip that lands at or past
 *    that limit also ends the chunk there.
 *  - skip_trigger >= 0xFFFFFFFF disables skipping (the paper's BASE
 *    ablation, Sec. VI-C).
 *  - Variant: with the ORACLE_SIGNED flag in `mode`, bytes are compared as
 *    signed (two's complement) values, as 8-bit signed vector compares would
 *    compare them (Sec. III-D's intrinsics); the reading above is unsigned.
 * Parity is pinned by hand-worked byte strings, closed forms, a mode
 * symmetry, brute force against a separately written bitmap-level
 * definition, invariants and exact expectations on random bytes.
 */
#include <stdint.h>

#define ORACLE_INCREASING 0u
#define ORACLE_DECREASING 1u
#define ORACLE_SIGNED 2u /* flag: bytes are signed values */

/* A byte's value under the mode: 0..255, or -128..127 with ORACLE_SIGNED. */
static int value(unsigned mode, uint8_t x) { return (mode & ORACLE_SIGNED) ? (int)(int8_t)x : (int)x; }

/* Target order (Sec. III-A "Modes of operation"): in Increasing mode a pair
 * (x, y) of neighbouring bytes is favourable when y > x and opposing when
 * y < x; Decreasing mode swaps the two. */
static int favourable(unsigned mode, uint8_t x, uint8_t y) {
  const int vx = value(mode, x), vy = value(mode, y);
  return (mode & ORACLE_DECREASING) == 0 ? (vy > vx) : (vy < vx);
}
static int opposing(unsigned mode, uint8_t x, uint8_t y) {
  const int vx = value(mode, x), vy = value(mode, y);
  return (mode & ORACLE_DECREASING) == 0 ? (vy < vx) : (vy > vx);
}

/*
 * Chunk b[0..n) and write the exclusive end offset of every chunk to
 * cuts[0..cap).  Returns the number of chunks (which may exceed cap: the
 * extra ends are not written), or -1 on invalid parameters.
 */
int64_t oracle_chunk(const uint8_t *b, uint64_t n, unsigned mode, unsigned seq_length, uint64_t min_size,
                     uint64_t max_size, uint64_t skip_trigger, uint64_t skip_size, uint64_t *cuts, uint64_t cap) {
  if (mode > 3 || seq_length < 2 || min_size < seq_length || max_size < min_size || skip_trigger < 1) return -1;
  int skipping = skip_trigger < 0xFFFFFFFFull;
  uint64_t count = 0;
  uint64_t c = 0; /* start of the current chunk */
  while (c < n) {
    /* Sec. IV: a chunk never grows past max_size; the stream end also ends it. */
    uint64_t limit = (n - c > max_size) ? c + max_size : n;
    /* Sec. III-B: the first min_size - SeqLength bytes are not scanned. */
    uint64_t s = c + min_size - seq_length;
    uint64_t cut = 0;
    for (;;) {
      /* One scan from s with fresh counters.  The run counter holds the
       * length (in bytes) of the monotone run ending at the current byte. */
      uint64_t run = 1, opp = 0;
      int skipped = 0;
      for (uint64_t j = s + 1; j < limit; j++) {
        uint8_t x = b[j - 1], y = b[j];
        if (favourable(mode, x, y)) {
          run++;
          if (run == seq_length) { /* Sec. III-A: boundary at the run's end */
            cut = j + 1;
            break;
          }
        } else {
          run = 1;
          if (opposing(mode, x, y)) {
            opp++;
            if (skipping && opp == skip_trigger) { /* Sec. III-C: unfavourable region */
              s = j + 1 + skip_size;             /* ignore the next skip_size bytes */
              skipped = 1;
              break;
            }
          }
        }
      }
      if (cut) break;
      if (!skipped || s >= limit) { /* nothing found before the limit */
        cut = limit;
        break;
      }
    }
    if (count < cap) cuts[count] = cut;
    count++;
    c = cut;
  }
  return (int64_t)count;
}

/*
 * The per-byte facts the vector formulation works from (Sec. III-D), as
 * bitmaps with bit (q mod 64) of word q/64 describing byte q:
 *   O[q] = 1 iff q >= 1 and (b[q-1], b[q]) is an opposing pair (mask M3);
 *   E[q] = 1 iff q >= SeqLength-1 and the SeqLength bytes b[q-SeqLength+1..q]
 *          are strictly monotone in the target order (the AND of the
 *          SeqLength-1 pairwise masks), i.e. a candidate run ends at q.
 * words = ceil(n / 64); bits at q >= n are zero.
 */
int oracle_mark(const uint8_t *b, uint64_t n, unsigned mode, unsigned seq_length, uint64_t *E, uint64_t *O) {
  if (mode > 3 || seq_length < 2) return -1;
  uint64_t words = (n + 63) / 64;
  for (uint64_t w = 0; w < words; w++) E[w] = O[w] = 0;
  for (uint64_t q = 1; q < n; q++)
    if (opposing(mode, b[q - 1], b[q])) O[q / 64] |= 1ull << (q % 64);
  for (uint64_t q = seq_length - 1; q < n; q++) {
    int all = 1;
    for (uint64_t i = q - seq_length + 2; i <= q; i++)
      if (!favourable(mode, b[i - 1], b[i])) {
        all = 0;
        break;
      }
    if (all) E[q / 64] |= 1ull << (q % 64);
  }
  return 0;
}
