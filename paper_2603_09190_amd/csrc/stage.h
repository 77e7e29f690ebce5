// Multi-stage staging of MFMA operands through LDS with direct global-to-LDS loads.
//
// global_load_lds_dwordx4 (gfx950) moves 16 bytes per lane from any global address straight into
// LDS at the wavefront-uniform base plus 16 x lane, without passing through VGPRs: one
// instruction fills one contiguous kilobyte of LDS.  A kernel keeps several K steps of its
// operands in flight this way and waits, once per step, only for the oldest step's loads (the
// load counter is in order, so a wait for step s leaves every later step in flight).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zp {

// 16 bytes per lane from gsrc (this lane's address) into LDS at base + 16 lane.
__device__ __forceinline__ void g2l16(const void* gsrc, void* lds_base) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)gsrc,
                                   (void __attribute__((address_space(3)))*)lds_base, 16, 0, 0);
}

// s_waitcnt with vmcnt <= N and no wait on the other counters (gfx9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Workgroup barrier that orders LDS accesses (outstanding global loads stay in flight).
__device__ __forceinline__ void lds_barrier_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace zp
