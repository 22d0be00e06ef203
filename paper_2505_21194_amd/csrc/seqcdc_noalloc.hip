// Allocation-free plain chunking: the path of seqcdc_chunk (mark, pass A
// chains, pass B continuations, stitch, compaction) with every workspace
// carved from one fixed device array that the library holds per GPU, and the
// single-file tables written there by a setup kernel, so a call allocates
// nothing, copies nothing from the host and waits for nothing.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/seqcdc.h"
#include "seqcdc_device.h"
#include "seqcdc_launch.h"
#include "seqcdc_runtime.h"

namespace seqcdc {

constexpr u64 kScratchBytes = SEQCDC_NOALLOC_SCRATCH_BYTES;
constexpr u32 kNoAllocSpanBlocks = 16;  // mark span: 16 KiB
constexpr u32 kNoAllocWaves = 8;        // chain waves per compute unit
constexpr int kMaxDevices = 64;

// The workspace of every allocation-free call on this GPU.  Host code never
// uses this name as an address: it holds the device address that
// hipGetSymbolAddress returns for the current device (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Identity tables of one file cut into nchains segments: chain -> file 0,
// list and continuation offsets, the chain order (pass A, pass B and
// compaction all take chains 0, 1, ...), the multi-segment file list {0}, the
// span hint table (every span is in file 0); clears the two work counters.
__global__ __launch_bounds__(256) void noalloc_setup_kernel(FileDesc fd, FileDesc* files, u32* hint, u32 nhint,
                                                            u32* chain_file, u64* list_off, u64* cont_off,
                                                            u32* iota, u32* multi, u32* heads, u32 nchains,
                                                            u64 list_per_chain, u32 cont_cap) {
  const u32 t = blockIdx.x * 256 + threadIdx.x;
  const u32 stride = gridDim.x * 256;
  if (t == 0) {
    files[0] = fd;
    multi[0] = 0;
  }
  for (u32 i = t; i < 32; i += stride) heads[i] = 0;
  for (u32 i = t; i < nhint; i += stride) hint[i] = 0;
  for (u32 c = t; c < nchains; c += stride) {
    chain_file[c] = 0;
    list_off[c] = (u64)c * list_per_chain;
    cont_off[c] = (u64)c * cont_cap;
    iota[c] = c;
  }
}

static std::mutex g_mu;
static unsigned char* g_ptr[kMaxDevices];  // device address of `scratch` on each device (null: not yet looked up)
static u32 g_cus[kMaxDevices];

// The device address of this GPU's scratch array and its CU count, looked up
// once per device with that device current.
static int scratch_ptr(unsigned char** ptr, u32* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SEQCDC_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    g_cus[dev] = n > 0 ? (u32)n : 1u;
    g_ptr[dev] = (unsigned char*)p;
  }
  *ptr = g_ptr[dev];
  *cus = g_cus[dev];
  return SEQCDC_OK;
}

// Bump allocation inside the scratch array (256-byte aligned pieces).
struct Carver {
  u64 off = 0;
  u64 take(u64 bytes) {
    off = (off + 255) & ~255ull;
    const u64 r = off;
    off += bytes;
    return r;
  }
};

}  // namespace seqcdc

using namespace seqcdc;

extern "C" int seqcdc_chunk_noalloc(const void* d_stream, uint64_t n, const seqcdc_params* p, uint64_t* d_cuts,
                                    uint64_t cap, uint64_t* d_count, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!d_count) return fail(SEQCDC_EINVAL, "d_count is NULL");
  if (n && !d_stream) return fail(SEQCDC_EINVAL, "d_stream is NULL");
  if (!d_cuts && cap) return fail(SEQCDC_EINVAL, "d_cuts is NULL");
  if (n >= kMaxStream) return fail(SEQCDC_EINVAL, "streams must be shorter than 256 GiB");
  // Segments as the plain path's defaults: 128 x min_size, at least 64 KiB,
  // whole mark spans.
  const u64 sb = (u64)kNoAllocSpanBlocks * kMarkBlock;
  u64 seg = 128 * p->min_size;
  if (seg < 64 * 1024) seg = 64 * 1024;
  if (n / seg > kMaxSegments) seg = n / kMaxSegments + 1;
  seg = (seg + sb - 1) / sb * sb;
  const u32 nseg = n > seg ? (u32)((n + seg - 1) / seg) : 1u;
  const u64 spans = (n + sb - 1) / sb;
  const u64 nhint = spans / kHintSpans + 2;
  const bool multi = nseg > 1;
  const u64 list_per_chain = seg / p->min_size + 2;
  u32 cont_cap = 64;
  if (multi) {
    const u64 want = 2 * seg / p->min_size + 64;
    cont_cap = (u32)(want < 1024 ? 1024 : want > 4096 ? 4096 : want);
  }

  // Layout of the scratch array for this call.
  Carver cv;
  const u64 o_files = cv.take(sizeof(FileDesc));
  const u64 o_hint = cv.take(nhint * 4);
  const u64 o_chain_file = cv.take(nseg * 4ull);
  const u64 o_list_off = cv.take(nseg * 8ull);
  const u64 o_cont_off = cv.take(nseg * 8ull);
  const u64 o_iota = cv.take(nseg * 4ull);
  const u64 o_multi = cv.take(4);
  const u64 o_heads = cv.take(32 * 4);
  const u64 o_list_cnt = cv.take(nseg * 4ull);
  const u64 o_conv_val = cv.take(nseg * 8ull);
  const u64 o_conv_chain = cv.take(nseg * 4ull);
  const u64 o_conv_idx = cv.take(nseg * 4ull);
  const u64 o_cont_cnt = cv.take(nseg * 8ull);
  const u64 o_ovf_start = cv.take(nseg * 8ull);
  const u64 o_ovf = cv.take(multi ? (n / p->min_size + 2) * 8 : 8);
  const u64 o_active = cv.take(nseg * 4ull);
  const u64 o_entry_idx = cv.take(nseg * 4ull);
  const u64 o_jumps = cv.take(nseg * 8ull);
  const u64 o_out_off = cv.take(nseg * 8ull);
  const u64 o_covered = cv.take(nseg * 8ull);
  const u64 o_list = cv.take(multi ? nseg * list_per_chain * 8 : 8);
  const u64 o_cont = cv.take(multi ? (u64)nseg * cont_cap * 8 : 8);
  const u64 o_eo = cv.take(16 * ((n + 63) / 64) + 256);
  const u64 o_esum = cv.take((((n + 1023) / 1024 + 15) & ~15ull) + 16 + 256);
  if (cv.off > kScratchBytes)
    return fail(SEQCDC_EINVAL,
                "seqcdc_chunk_noalloc: %llu bytes at min_size %llu need %llu bytes of workspace; the fixed scratch "
                "holds %llu",
                (unsigned long long)n, (unsigned long long)p->min_size, (unsigned long long)cv.off,
                (unsigned long long)kScratchBytes);
  unsigned char* base = nullptr;
  u32 cus = 1;
  if ((rc = scratch_ptr(&base, &cus))) return rc;
  hipStream_t st = (hipStream_t)stream;
  FileDesc fd{};
  fd.data = (const uint8_t*)d_stream;
  fd.n = n;
  fd.eo = (u32*)(base + o_eo);
  fd.esum = base + o_esum;
  fd.mode = p->mode;
  fd.sl = p->seq_length;
  fd.min_size = p->min_size;
  fd.max_size = p->max_size;
  fd.trig = p->skip_trigger;
  fd.skip = p->skip_size;
  fd.mark_span0 = 0;
  fd.seg = seg;
  fd.nseg = nseg;
  fd.chain0 = 0;
  fd.out = d_cuts;
  fd.out_cap = cap;
  fd.out_count = d_count;
  fd.ovf0 = 0;

  const FileDesc* d_files = (const FileDesc*)(base + o_files);
  u32* heads = (u32*)(base + o_heads);
  const u32 setup_groups = std::min<u32>(64, (nseg + 255) / 256);
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(setup_groups), dim3(256), 0, st, fd, (FileDesc*)d_files,
                     (u32*)(base + o_hint), (u32)nhint, (u32*)(base + o_chain_file), (u64*)(base + o_list_off),
                     (u64*)(base + o_cont_off), (u32*)(base + o_iota), (u32*)(base + o_multi), heads, nseg,
                     list_per_chain, cont_cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "noalloc_setup_kernel");

  ChainWs ws;
  ws.chain_file = (u32*)(base + o_chain_file);
  ws.list = (u64*)(base + o_list);
  ws.list_off = (u64*)(base + o_list_off);
  ws.list_cnt = (u32*)(base + o_list_cnt);
  ws.conv_val = (u64*)(base + o_conv_val);
  ws.conv_chain = (u32*)(base + o_conv_chain);
  ws.conv_idx = (i32*)(base + o_conv_idx);
  ws.cont_cnt = (u64*)(base + o_cont_cnt);
  ws.ovf_start = (u64*)(base + o_ovf_start);
  ws.ovf = (u64*)(base + o_ovf);
  ws.cont = (u64*)(base + o_cont);
  ws.cont_off = (u64*)(base + o_cont_off);
  ws.cont_cap = cont_cap;
  ws.active = (u32*)(base + o_active);
  ws.entry_idx = (i32*)(base + o_entry_idx);
  ws.out_off = (u64*)(base + o_out_off);
  ws.jumps = (u32*)(base + o_jumps);
  ws.covered = (u32*)(base + o_covered);

  const u32* iota = (const u32*)(base + o_iota);
  const u32 groups = cus * kNoAllocWaves / kWavesPerGroup;
  if ((e = launch_mark(d_files, (const u32*)(base + o_hint), 0, spans, kNoAllocSpanBlocks, st)) != hipSuccess)
    return hip_fail(e, "mark kernel");
  if ((e = launch_chains(d_files, ws, iota, nseg, heads, std::min<u32>(groups, (nseg + 3) / 4), false, st)) !=
      hipSuccess)
    return hip_fail(e, "chains kernel");
  if (multi) {
    const u32 nb = nseg - 1;
    if ((e = launch_continue(d_files, ws, iota, nb, heads + 16, std::max<u32>(1, std::min<u32>(groups, (nb + 3) / 4)),
                             false, st)) != hipSuccess)
      return hip_fail(e, "continue kernel");
    if ((e = launch_stitch(d_files, ws, (const u32*)(base + o_multi), 1, false, st)) != hipSuccess)
      return hip_fail(e, "stitch kernel");
    if ((e = launch_compact(d_files, ws, iota, nseg, st)) != hipSuccess) return hip_fail(e, "compact kernel");
  }
  return SEQCDC_OK;
}
