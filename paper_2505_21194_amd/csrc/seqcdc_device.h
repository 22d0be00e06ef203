// Wave-level device helpers shared by the mark and resolve kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "seqcdc_internal.h"

namespace seqcdc {

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Global-memory view of a pointer.  Pointers read from descriptors are
// generic, and generic accesses compile to FLAT instructions (64-bit VGPR
// addresses, counted by both the vector-memory and LDS/scalar counters);
// through this view they compile to global loads and stores.
#ifndef SEQCDC_GLOBAL
#define SEQCDC_GLOBAL __attribute__((address_space(1)))
#endif
template <class T>
__device__ __forceinline__ SEQCDC_GLOBAL T* as_global(T* p) {
  return (SEQCDC_GLOBAL T*)p;
}

// LDS view of a pointer into a __shared__ array.
#ifndef SEQCDC_LOCAL
#define SEQCDC_LOCAL __attribute__((address_space(3)))
#endif

// Waits until every vector-memory operation of the wave has completed,
// including LDS DMA writes (global_load_lds), which the compiler does not
// track; the memory clobber keeps LDS reads from moving above it.
#ifndef SEQCDC_WAIT_VMEM
#define SEQCDC_WAIT_VMEM() asm volatile("s_waitcnt vmcnt(0)" ::: "memory")
#endif

// 16-byte global load (HIP's uint4 class cannot be copied out of a
// global-address-space reference, a plain vector type can).
__device__ __forceinline__ uint4 load16(const void* p) {
  const u32x4 v = *as_global((const u32x4*)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}

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

// 64-bit inclusive prefix sum across the wave: the same DPP steps on both
// halves, with the carry out of the low half added to the high half.
__device__ __forceinline__ u64 wave_incl_scan64(u64 v) {
  u32 lo = (u32)v, hi = (u32)(v >> 32);
  auto step = [&](u32 slo, u32 shi) {
    const u32 nlo = lo + slo;
    hi += shi + (nlo < lo ? 1u : 0u);
    lo = nlo;
  };
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x111, 0xf, 0xf, true), __builtin_amdgcn_update_dpp(0u, hi, 0x111, 0xf, 0xf, true));
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x112, 0xf, 0xf, true), __builtin_amdgcn_update_dpp(0u, hi, 0x112, 0xf, 0xf, true));
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x114, 0xf, 0xf, true), __builtin_amdgcn_update_dpp(0u, hi, 0x114, 0xf, 0xf, true));
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x118, 0xf, 0xf, true), __builtin_amdgcn_update_dpp(0u, hi, 0x118, 0xf, 0xf, true));
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x142, 0xa, 0xf, false), __builtin_amdgcn_update_dpp(0u, hi, 0x142, 0xa, 0xf, false));
  step(__builtin_amdgcn_update_dpp(0u, lo, 0x143, 0xc, 0xf, false), __builtin_amdgcn_update_dpp(0u, hi, 0x143, 0xc, 0xf, false));
  return (u64)lo | ((u64)hi << 32);
}

// Takes the next index of a work counter for the whole wave.  Every lane
// executes the atomic (lane 0 adds 1, the others 0), so no branch surrounds it
// and the value lane 0 receives is read back in the same straight-line code.
__device__ __forceinline__ u32 wave_pop(u32* head) {
  const u32 v = atomicAdd(head, lane_id() == 0 ? 1u : 0u);
  return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace seqcdc
