// Host runtime internals of libseqcdc: plans, buffers, tuning cache.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/seqcdc.h"
#include "seqcdc_internal.h"
#include "seqcdc_workspace.h"

namespace seqcdc {

constexpr u64 kMaxSegments = 65536;  // per stream
constexpr u32 kMaxGroups = 8;        // file groups of an overlapped batch
constexpr u64 kMaxStream = 1ull << 38;  // 256 GiB: group and sub-window indices stay 32-bit

// Workspace (re)allocations made by DevBuf / HostBuf since the process
// started (each frees the old buffer: hipFree / hipHostFree synchronise).
u64 realloc_count();

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int reserve(size_t bytes);
  void release();
};

struct HostBuf {  // pinned
  void* p = nullptr;
  size_t cap = 0;
  int reserve(size_t bytes);
  void release();
};

struct TuneKey {
  std::string arch;
  u32 cus = 0, sl = 0;
  int avg_class = 0;
  bool operator==(const TuneKey& o) const {
    return arch == o.arch && cus == o.cus && sl == o.sl && avg_class == o.avg_class;
  }
};

struct TuneEntry {
  TuneKey key;
  u64 seg_mult = 128;  // segment length = seg_mult * min_size
  u32 span_blocks = 8;
  u32 waves_per_cu = 8;
  int mode = 0;
  double ms = 0;
  u64 sample = 0;  // bytes of the stream the choices were measured on
};

struct Plan {
  int device = 0;
  u32 cus = 256;
  std::string arch;
  std::mutex mu;
  DevBuf eo, esum, list, cont, chains, tables, flags, misc;
  DevBuf aux;        // calibration: candidates' cut lists and statistics
  DevBuf ovf;        // overflow regions of open continuations the stitch takes further
  HostBuf staging, readback, aux_host;
  hipEvent_t call_done = nullptr, upload_done = nullptr;
  bool pending = false, upload_pending = false;
  // the last tables uploaded, and the device buffer (address, capacity) they
  // went to: a call whose staged tables are the same bytes skips the copy
  std::vector<char> uploaded;
  const void* uploaded_dev = nullptr;
  size_t uploaded_cap = 0;
  hipStream_t last_stream = nullptr;
  u32 last_nchains = 0, last_multi = 0;
  u64 seg_override = 0;
  u32 span_override = 0, waves_override = 0;
  int mode = -1;  // resolve mode (0: marked, 1: direct); -1: tuned (else 0)
  // optional per-phase timing of the last call: events before the mark
  // kernel and after the mark, pass A, pass B and stitch + compaction
  bool timing = false, timed = false;
  hipEvent_t tev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // overlapped batches: files in groups, largest first; the mark kernels of
  // later groups run on the caller's stream while side[0] runs the chains of
  // earlier ones and side[1] their continuations
  u32 overlap = 0;  // groups (0: default, 1: off)
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t ev_mark[kMaxGroups] = {};
  hipEvent_t ev_chain_first = nullptr, ev_chain_last = nullptr, ev_join = nullptr;

  u64 segment_for(u64 n, const seqcdc_params* p, bool single) const;
  u32 span_blocks_for(const seqcdc_params* p) const;
  u32 waves_for(const seqcdc_params* p) const;
  int mode_for(const seqcdc_params* p) const;
  u32 groups_for(u32 nfiles, u64 total) const;
  // set while a prepared batch captures its launch sequence: no uploads, host
  // waits or bookkeeping events (the tables are already on the device)
  bool capturing = false;
};

// A stream of a batch, before device pointers are assigned.
struct Spec {
  const uint8_t* data;
  u64 n;
  const seqcdc_params* p;
  u64* out;
  u64 out_cap;
  u64* out_count;
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate(const seqcdc_params* p);
u64 max_cuts(u64 n, const seqcdc_params* p);
int plan_init(Plan* pl, int device);
void plan_free(Plan* pl);
int chunk_plan(Plan* pl, const void* d_stream, u64 n, const seqcdc_params* p, u64* d_cuts, u64 cap, u64* h_count,
               hipStream_t st);
int chunk_batch(Plan* pl, const seqcdc_file* files, u32 nfiles, const seqcdc_params* params, u32 nparams,
                u64* d_cuts, const u64* h_off, u64* d_counts, hipStream_t st);
int build_specs(const seqcdc_file* files, u32 nfiles, const seqcdc_params* params, u32 nparams, u64* d_cuts,
                const u64* h_off, u64* d_counts, std::vector<Spec>& specs);
int run_batch(Plan* pl, const Spec* specs, u32 nfiles, hipStream_t st, bool mark_only);
int plan_reserve(Plan* pl, u64 bytes, u32 nfiles, const seqcdc_params* params, u32 nparams, bool dry, u64* total);
TuneKey plan_key(const Plan* pl, const seqcdc_params* p);
bool tune_lookup(const TuneKey& k, TuneEntry* out);
void tune_store(const TuneEntry& e);

}  // namespace seqcdc
