/*
 * libseqcdc -- SeqCDC chunk-boundary detection on AMD Instinct MI355X (gfx950).
 *
 * SeqCDC (Udayashankar & Al-Kiswany, "Vectorized Sequence-Based Chunking for
 * Data Deduplication", arXiv 2505.21194) cuts a byte stream into chunks:
 *   - a chunk ends just after the first run of seq_length bytes that is
 *     strictly increasing (Increasing mode) or strictly decreasing
 *     (Decreasing mode)                                       [Sec. III-A]
 *   - the first min_size - seq_length bytes of every chunk are not scanned,
 *     so no chunk (except the last) is shorter than min_size  [Sec. III-B]
 *   - after skip_trigger pairs of bytes in the opposing order, the next
 *     skip_size bytes are not scanned and the counters restart [Sec. III-C]
 *   - a chunk ends at max_size bytes if no run is found       [Sec. IV]
 * Bytes are unsigned; comparisons are strict (an equal pair ends a run and is
 * not opposing).  A boundary is reported as the exclusive end offset of its
 * chunk: chunks are [0, cuts[0]), [cuts[0], cuts[1]), ... and the last cut is
 * the stream length.  An empty stream has no cuts.  At most
 * floor(n / min_size) + 1 cuts are produced for n bytes.
 *
 * Conventions for every call:
 *   - "d_" pointers are device (HBM) pointers of the current HIP device,
 *     "h_" pointers are host pointers.  The caller owns every buffer passed
 *     in; the library never frees them.  Inputs may have any alignment.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Return value 0 on success, a negative SEQCDC_E* code on failure.
 *     seqcdc_last_error() describes the most recent failure of the calling
 *     thread.  No C++ exception or abort crosses this interface.
 */
#ifndef SEQCDC_H
#define SEQCDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEQCDC_OK 0
#define SEQCDC_EINVAL (-1)    /* bad parameters or NULL pointers */
#define SEQCDC_ECAPACITY (-2) /* output too small; *h_count holds the required count */
#define SEQCDC_EHIP (-3)      /* a HIP runtime call failed */
#define SEQCDC_EBUDGET (-4)   /* serving: request larger than the memory budget */
#define SEQCDC_ENOMEM (-5)    /* host or device allocation failed */
#define SEQCDC_EAGAIN (-6)    /* serving: result not ready yet */
#define SEQCDC_ENOENT (-7)    /* serving: unknown ticket */

#define SEQCDC_INCREASING 0u /* Sec. III-A "Modes of operation" */
#define SEQCDC_DECREASING 1u
#define SEQCDC_SIGNED 2u /* mode flag: compare bytes as signed (two's complement) values, as the 8-bit signed
                            vector compares of Sec. III-D would; the default reading is unsigned */
#define SEQCDC_NO_SKIP 0xFFFFFFFFu /* skip_trigger value that disables content-based skipping */

/* SeqCDC parameters (Sec. III; Table I; min/max rule of Sec. VI). */
typedef struct {
  uint32_t mode;         /* SEQCDC_INCREASING or SEQCDC_DECREASING, optionally | SEQCDC_SIGNED */
  uint32_t seq_length;   /* bytes in the monotone run, 2..16 */
  uint64_t min_size;     /* >= seq_length */
  uint64_t max_size;     /* >= min_size, <= 1 GiB */
  uint32_t skip_trigger; /* opposing pairs that trigger a skip, >= 1; SEQCDC_NO_SKIP disables */
  uint32_t skip_size;    /* bytes not scanned after the trigger byte */
} seqcdc_params;

/* Validate a parameter set: 0 or SEQCDC_EINVAL. */
int seqcdc_params_validate(const seqcdc_params* p);

/* Parameters for a target average chunk size (Increasing mode).  Table I gives
 * SeqLength 5 with SkipTrigger/SkipSize 55/256, 50/256 and 50/512 for 4, 8 and
 * 16 KiB; Sec. VI uses min = avg/2 (1 KiB at 4 KiB) and max = 2*avg.  Larger
 * averages keep 50/512.  avg must be a power of two >= 4096. */
int seqcdc_params_for_avg(uint64_t avg, seqcdc_params* out);

/* Upper bound on the number of cuts for n bytes: floor(n / min_size) + 1 (0 for n = 0). */
uint64_t seqcdc_max_cuts(uint64_t n, const seqcdc_params* p);

/* Plans own device workspaces (mark bitmaps: n/4 bytes per n input bytes,
 * plus per-segment cut lists), pinned staging memory and tuning choices.  A
 * plan grows on demand.  Calls on one plan must not overlap: the library
 * waits for the plan's previous call when a call arrives on another stream.
 * device: HIP device ordinal, or -1 for the current device. */
typedef struct seqcdc_plan seqcdc_plan;
int seqcdc_plan_create(int device, seqcdc_plan** out);
int seqcdc_plan_destroy(seqcdc_plan* plan);

/* Tuning knobs of a plan (0 = keep).  segment_bytes: length of the segments
 * a stream is split into for speculative resolution (rounded up to a whole
 * number of mark spans; default: the autotuner's choice, used as it is on
 * streams of at least half the size it was measured on, else 128 x min_size;
 * on other single streams it shrinks down to the stream's bytes divided by
 * the device's chain waves (CUs x waves_per_cu), but not below
 * 64 KiB x (min_size / 4 KiB)^2; at least 64 KiB);
 * mark_span_blocks: 1 KiB blocks per mark span, the
 * unit of marking work (4, 8, 16, 32 or 64); waves_per_cu: waves per compute
 * unit of the persistent chain kernels, one chain per wave (4..32, a
 * multiple of 4; default 8; each wave keeps 8 KiB of windows in LDS, so at
 * most 20 are resident per compute unit). */
int seqcdc_plan_set_tuning(seqcdc_plan* plan, uint64_t segment_bytes, uint32_t mark_span_blocks,
                           uint32_t waves_per_cu);
/* Current choices for a stream of n bytes under p. */
int seqcdc_plan_get_tuning(seqcdc_plan* plan, uint64_t n, const seqcdc_params* p, uint64_t* segment_bytes,
                           uint32_t* mark_span_blocks, uint32_t* waves_per_cu);

/* How a plan runs the resolve stage.  0 (marked, the default): the mark
 * kernel writes run-end and opposing bits for every input byte, then pass A
 * (chains) and pass B (continuations) walk them.  1 (direct, skip-aware): no
 * mark kernel; each chain loads the raw bytes of the 1 KiB windows it scans
 * and computes their bits itself, so the sub-minimum region after every cut
 * and the bytes a skip passes over are never read (Sec. III-B, III-C).
 * Overlapped batches are marked-mode only.  All modes give the same cuts. */
int seqcdc_plan_set_mode(seqcdc_plan* plan, int mode);

/* Overlapped batches (mode 0 only): the files of a seqcdc_chunk_batch call
 * are taken largest first and cut into groups.  The caller's stream marks one
 * group after the other while two side streams of the plan (default
 * priority) run the chains of each group as soon as its marks are done, the
 * continuations of the first group as soon as its chains are done, then the
 * remaining continuations, stitch and compaction; the caller's stream waits
 * for them before the call's work counts as done.  0 = default (off: back
 * to back, or with several serving passes in flight, the side streams cost
 * more than the overlap gains on MI355X); 1 = off; 2 = two groups, the files
 * with more than one segment (whose continuations are the long part of
 * resolve) and the others (equal byte shares if the batch has one kind
 * only), which shortens a single synchronous call by about 5 %; up to 8 =
 * groups of about equal bytes.  Results do not depend on it.  Prepared
 * batches (below) do not overlap. */
int seqcdc_plan_set_overlap(seqcdc_plan* plan, uint32_t groups);

/* Per-phase timing of the plan's calls (off by default; on adds HIP events
 * to every call).  seqcdc_plan_phase_ms waits for the plan's last timed call
 * and writes 4 durations in milliseconds: the mark kernel (events right
 * before and after its launch), pass A (speculative chains), pass B
 * (continuations), stitch + compaction.  Overlapped batches: the marking of
 * all groups on the caller's stream, then what each later step added after
 * the previous one ended (chains of the last group, the continuations, stitch
 * + compaction).  The values after the first are 0 when no stream had more
 * than one segment.  SEQCDC_EINVAL if no timed call was made. */
int seqcdc_plan_set_timing(seqcdc_plan* plan, int on);
int seqcdc_plan_phase_ms(seqcdc_plan* plan, float* ms4);

/* Autotuner: time candidate segment sizes, mark spans, resolve occupancies and
 * both resolve modes on the given device-resident sample stream (the best of
 * 3 calls each, then the 3 fastest again over 10 calls), and keep
 * the fastest in a process-wide cache keyed by (arch, CU count, seq_length,
 * average class), which plans consult for settings not set explicitly.
 * Results are exact for every choice; only speed differs.  *best_ms receives
 * the best time (may be NULL). */
int seqcdc_autotune(seqcdc_plan* plan, const void* d_sample, uint64_t n, const seqcdc_params* p, double* best_ms,
                    void* stream);

/* Chunk one device-resident stream (the plain path).
 * d_stream: n bytes, n < 256 GiB (SEQCDC_EINVAL otherwise; the same limit
 * holds per file in seqcdc_chunk_batch and for seqcdc_mark).  d_cuts: room for `cap` uint64 cut offsets.  On return
 * *h_count is the number of cuts; if it exceeds cap the call returns
 * SEQCDC_ECAPACITY and only the first cap cuts were written.  Synchronous:
 * the cuts are in d_cuts when it returns.  plan may be NULL (a per-device
 * library plan is used). */
int seqcdc_chunk(const void* d_stream, uint64_t n, const seqcdc_params* p, uint64_t* d_cuts, uint64_t cap,
                 uint64_t* h_count, void* stream);
int seqcdc_chunk_plan(seqcdc_plan* plan, const void* d_stream, uint64_t n, const seqcdc_params* p, uint64_t* d_cuts,
                      uint64_t cap, uint64_t* h_count, void* stream);

/* One file of a batch. */
typedef struct {
  const void* d_data;    /* device pointer to the file's bytes */
  uint64_t n;            /* length in bytes */
  uint32_t params_index; /* index into the batch's params array */
  uint32_t reserved;     /* must be 0 */
} seqcdc_file;

/* Chunk many independent device-resident files in one pass: one mark launch
 * over all files, one persistent launch of speculative chains over every
 * (file, segment) (largest first), then continuations, stitching and
 * compaction.
 * h_cut_offsets: host array of nfiles+1 offsets; file f's cuts go to
 *   d_cuts[h_cut_offsets[f] ..], and each range must hold at least
 *   seqcdc_max_cuts(n_f, params) entries (checked; SEQCDC_EINVAL otherwise).
 * d_counts: device array of nfiles uint64 counts (written).
 * Asynchronous: results are ready once `stream` reaches the end of the call. */
int seqcdc_chunk_batch(seqcdc_plan* plan, const seqcdc_file* h_files, uint32_t nfiles, const seqcdc_params* h_params,
                       uint32_t nparams, uint64_t* d_cuts, const uint64_t* h_cut_offsets, uint64_t* d_counts,
                       void* stream);

/* Autotuner for a batch: times candidate segment lengths (multiples of the
 * smallest min_size), mark spans, chain occupancies and both resolve modes on
 * seqcdc_chunk_batch itself with the given arguments (as for that call; the
 * best of 3 calls each, then the 3 fastest again over 10 calls), and
 * sets the fastest as the plan's own settings (those seqcdc_plan_set_tuning
 * and seqcdc_plan_set_mode set; they replace earlier ones and take precedence
 * over the process-wide cache).  The best settings for many files differ from
 * those for one stream of the same parameters.  Synchronous; the batch's
 * outputs hold its results when it returns.  Results are exact for every
 * choice; only speed differs.  *best_ms receives the best time (may be NULL).
 * Errors as for seqcdc_chunk_batch; SEQCDC_EINVAL for an empty batch. */
int seqcdc_autotune_batch(seqcdc_plan* plan, const seqcdc_file* h_files, uint32_t nfiles, const seqcdc_params* h_params,
                          uint32_t nparams, uint64_t* d_cuts, const uint64_t* h_cut_offsets, uint64_t* d_counts,
                          double* best_ms, void* stream);

/* Prepared batches, for callers that chunk the same set of device buffers
 * again and again (a ring of staging buffers refilled with new data, a fixed
 * set of volumes).  seqcdc_batch_prepare lays the batch out once, in a
 * workspace the batch owns, runs it once (synchronously), and captures its
 * launch sequence (kernels only: counter clearing, mark, pass A, pass B,
 * stitch, compaction) into a hipGraph.  seqcdc_batch_launch replays the graph
 * on `stream`: the files' current contents are chunked into the same d_cuts /
 * d_counts, with no host-side work beyond the graph launch; the results are
 * those seqcdc_chunk_batch gives.  Arguments are those of seqcdc_chunk_batch
 * and stay owned by the caller; the file pointers, lengths, parameters and
 * output arrays are fixed at preparation and must stay valid until the batch
 * is destroyed.  `settings` (may be NULL) supplies tuning choices and the
 * resolve mode; overlapped groups are not used.  Launches of one batch run
 * one after the other, whatever their streams (each waits for the previous
 * one).  seqcdc_batch_destroy waits for the last launch.  Errors as for
 * seqcdc_chunk_batch; nfiles must be at least 1. */
typedef struct seqcdc_batch seqcdc_batch;
int seqcdc_batch_prepare(seqcdc_plan* settings, const seqcdc_file* files, uint32_t nfiles,
                         const seqcdc_params* params, uint32_t nparams, uint64_t* d_cuts,
                         const uint64_t* h_cut_offsets, uint64_t* d_counts, seqcdc_batch** out);
int seqcdc_batch_launch(seqcdc_batch* batch, void* stream);
int seqcdc_batch_destroy(seqcdc_batch* batch);

/* The mark step alone (Sec. III-D masks), for inspection and tests.
 * d_eo receives 4 * ceil(n/64) uint32 words: byte q belongs to group q/64;
 * word 4g+j holds, for the 16 bytes 64g+16j .. 64g+16j+15 (bit i = byte
 * 64g+16j+i), the run-end bits E in bits 0..15 and the opposing-pair bits O in
 * bits 16..31.  E marks bytes that end a run of seq_length strictly monotone
 * bytes; O marks bytes smaller (Increasing) / larger (Decreasing) than their
 * predecessor.  Asynchronous. */
int seqcdc_mark(const void* d_stream, uint64_t n, const seqcdc_params* p, uint32_t* d_eo, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * path of seqcdc_chunk with every workspace (mark bitmaps, per-segment cut
 * lists, continuation buffers, chain state, tables, work counters) carved from
 * one fixed device array of SEQCDC_NOALLOC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends.  The call allocates
 * nothing (no hipMalloc, hipHostMalloc or frees), copies nothing from the
 * host and does not wait: it only enqueues kernels on `stream`, the first of
 * which writes this call's tables and clears its counters.  Results are those
 * of seqcdc_chunk (same segment length rule, 128 x min_size, at least
 * 64 KiB; the autotuner's choices are not consulted).
 * d_count: device pointer receiving the number of cuts; if it exceeds cap,
 *   only the first cap cuts were written to d_cuts.
 * Errors: SEQCDC_EINVAL for bad arguments and for streams whose workspace
 *   (about n/4 + n/64 bytes at the Table I parameters, so up to about 230 MiB
 *   of input) does not fit the scratch array; the message gives both sizes.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (on different streams, or from several threads, without ordering between
 * them) race and give wrong results. */
#define SEQCDC_NOALLOC_SCRATCH_BYTES (64ull << 20)
int seqcdc_chunk_noalloc(const void* d_stream, uint64_t n, const seqcdc_params* p, uint64_t* d_cuts, uint64_t cap,
                         uint64_t* d_count, void* stream);

/* Host convenience: copy h_stream to the device, chunk it, copy the cuts back. */
int seqcdc_chunk_host(const uint8_t* h_stream, uint64_t n, const seqcdc_params* p, uint64_t* h_cuts, uint64_t cap,
                      uint64_t* h_count);

/* Space savings of exact-content deduplication (Eq. 1) over the chunks of
 * several host buffers: chunk i of buffer b is [cuts_b[i-1], cuts_b[i]).
 * Outputs original bytes, unique bytes, savings = (orig - unique) / orig and
 * ratio = orig / unique.  Chunks are matched by a 128-bit hash and confirmed
 * byte for byte. */
int seqcdc_dedup_stats(const uint8_t* const* h_buffers, const uint64_t* const* h_cut_lists, const uint64_t* h_counts,
                       uint32_t nbuffers, uint64_t* orig_bytes, uint64_t* unique_bytes, double* savings,
                       double* ratio);

/* Monte-Carlo calibration (Sec. V, Table I): the paper chooses SeqLength,
 * SkipTrigger and SkipSize so that random data gives the target average chunk
 * size.  seqcdc_calibrate chunks the device-resident sample (n bytes, normally
 * uniform random bytes the caller generated) under each of the ncand candidate
 * parameter sets, all in one batched call, and reduces each candidate's chunk
 * statistics on the device into out[i].  Synchronous; uses the plan's
 * workspace (about 8 x n / min_size bytes per candidate for the cut lists). */
typedef struct {
  uint64_t chunks;     /* chunks of the sample (the last one included) */
  uint64_t max_chunks; /* chunks cut at max_size, the last chunk not counted */
  double mean;         /* n / chunks */
  double stddev;       /* of the chunk lengths */
} seqcdc_calib_stats;
int seqcdc_calibrate(seqcdc_plan* plan, const void* d_sample, uint64_t n, const seqcdc_params* cands, uint32_t ncand,
                     seqcdc_calib_stats* out, void* stream);

/* Deduplication on the device, the stage after chunking (Sec. II, Eq. 1):
 * the chunks of many device-resident files, laid out as seqcdc_chunk_batch
 * writes them (file f's cuts at d_cuts[h_cut_offsets[f] ..], d_counts[f] of
 * them, chunk i = [cut i-1, cut i) with cut -1 = 0), are fingerprinted with
 * SHA-256 (FIPS 180-4), entered into an open-addressing table of
 * fingerprints, and every chunk whose fingerprint is already in the table is
 * compared byte for byte with the chunk that holds the entry.  Outputs: the
 * original bytes (all chunks) and the unique bytes (chunks that are not a
 * byte-for-byte copy of an earlier entry), so savings = (orig - unique) /
 * orig and ratio = orig / unique.  d_digests (may be NULL): receives the
 * fingerprint of the chunk in cut slot s at d_digests[8 (s - h_cut_offsets[0])
 * ..], eight 32-bit words, word 0 first, each the big-endian word of the
 * standard's digest (slots past a file's count get zeros).  The plan provides
 * the workspace (the table has at least twice as many entries as cut slots)
 * and must not be used by another call at the same time.  seqcdc_file's
 * params_index is ignored.  Synchronous. */
int seqcdc_dedup_batch(seqcdc_plan* plan, const seqcdc_file* h_files, uint32_t nfiles, const uint64_t* d_cuts,
                       const uint64_t* h_cut_offsets, const uint64_t* d_counts, uint32_t* d_digests,
                       uint64_t* h_orig, uint64_t* h_unique, void* stream);

/* ---------------------------------------------------------------------
 * Serving: a dedup-ingest request loop with continuous batching.
 * Requests reference device-resident bytes.  The memory budget is split
 * evenly between `streams` passes; at creation each pass reserves, once, the
 * workspace for the largest group of requests its share can hold (its input
 * capacity plus that workspace fit the share), so admission and passes never
 * allocate or free.  A scheduler thread admits queued requests into a free
 * pass while their bytes fit its capacity and a ring slot is free, launches
 * each admitted group as one batched pass on the pass's HIP stream (groups
 * overlap on the GPU), and publishes each request's cuts and latency when its
 * pass completes.  The oldest queued request is never overtaken.  When
 * several passes are free, each takes an equal share of the queued bytes, so
 * a backlog runs as passes in flight together.
 * Passes use the phased resolve launches without overlapped groups and 8
 * chain waves per compute unit; segment length and mark span follow the
 * autotuner's choices, if any. 
 * ------------------------------------------------------------------- */
typedef struct {
  int device;                /* -1 = current */
  uint64_t budget_bytes;     /* in-flight input bytes plus the passes' workspaces (reserved at creation) */
  uint32_t ring_slots;       /* max requests in flight */
  uint32_t streams;          /* concurrent batched passes (1..8) */
  uint32_t max_batch;        /* max requests per pass */
  uint32_t nparams;          /* parameter sets requests may use */
  const seqcdc_params* params;
} seqcdc_server_config;

typedef struct {
  int32_t status;      /* 0 done, SEQCDC_EAGAIN pending, or an error code */
  uint32_t reserved;
  uint64_t count;      /* number of cuts */
  const uint64_t* cuts; /* host memory owned by the server, valid until seqcdc_server_release(ticket) */
  double latency_ms;   /* submit -> cuts available on the host */
  double queue_ms;     /* submit -> admission */
} seqcdc_result;

typedef struct seqcdc_server seqcdc_server;
int seqcdc_server_create(const seqcdc_server_config* cfg, seqcdc_server** out);
/* Queue a request; *ticket identifies it.  SEQCDC_EBUDGET if it is larger
 * than one pass can hold (budget / streams less that pass's workspace). */
int seqcdc_server_submit(seqcdc_server* s, const void* d_data, uint64_t n, uint32_t params_index, uint64_t* ticket);
/* Queue n requests (d_data, n and params_index of each seqcdc_file; reserved
 * must be 0) from one call, each with its own ticket, as n separate submits
 * would.  at_ms == NULL: all at once.  Otherwise request i is queued at_ms[i]
 * milliseconds after the call starts (non-decreasing offsets; the call
 * returns after the last one), which replays an arrival process at rates a
 * caller's own loop could not reach.  submitted_ms (may be NULL) receives
 * when each request was queued, in milliseconds after the call started.
 * Every request is validated first: on an error nothing is queued. */
int seqcdc_server_submit_many(seqcdc_server* s, const seqcdc_file* reqs, uint32_t n, const double* at_ms,
                              uint64_t* tickets, double* submitted_ms);
/* Non-blocking: fills *out; returns 0 when done, SEQCDC_EAGAIN while pending. */
int seqcdc_server_poll(seqcdc_server* s, uint64_t ticket, seqcdc_result* out);
/* Block until the ticket is done (timeout_ms < 0: no limit). */
int seqcdc_server_wait(seqcdc_server* s, uint64_t ticket, double timeout_ms, seqcdc_result* out);
/* Free the host copy of a finished request's cuts. */
int seqcdc_server_release(seqcdc_server* s, uint64_t ticket);
/* Counters: requests admitted, passes launched, peak bytes (input bytes in
 * flight plus the passes' reserved workspaces; never above the budget), peak
 * requests in flight. */
int seqcdc_server_stats(seqcdc_server* s, uint64_t* admitted, uint64_t* passes, uint64_t* peak_bytes,
                        uint64_t* peak_inflight);

/* One batched pass of the serving loop, for diagnosing throughput. */
typedef struct {
  uint32_t requests;  /* requests in the pass */
  uint32_t grew;      /* workspace buffers (re)allocated while the pass was laid out (each frees the old one) */
  uint64_t bytes;     /* input bytes */
  double wait_ms;     /* admission -> the scheduler starts laying the pass out */
  double layout_ms;   /* host: tables laid out and every launch and copy of the pass enqueued */
  double gpu_ms;      /* device: the pass's work on its stream, kernels and result copies (HIP events) */
  double retire_ms;   /* enqueue done -> the scheduler saw the pass complete and published its results */
} seqcdc_pass_record;
/* The most recent passes (up to 4096 are kept), oldest first: writes up to
 * cap records to out and their number to *count. */
int seqcdc_server_timeline(seqcdc_server* s, seqcdc_pass_record* out, uint32_t cap, uint32_t* count);
int seqcdc_server_destroy(seqcdc_server* s);

/* Description of the calling thread's most recent failure ("" if none). */
const char* seqcdc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEQCDC_H */
