// Device helpers shared by the kernels that stream operands through LDS rings with
// direct-to-LDS loads (included by HIP sources only).
#pragma once
#include <hip/hip_runtime.h>

namespace lrs {

// Workgroup barrier of the LDS ring.  __syncthreads() carries a release fence, for which the
// compiler drains every direct-to-LDS load in flight; here each wave retires exactly what the
// next step needs instead: its own LDS reads (so a slot may be refilled) and its global->LDS
// loads up to the last KEEP (loads complete in order, so with only loads in flight this means
// every load but the last KEEP has landed).  The empty asm statements with a memory clobber
// keep the compiler from moving memory accesses across the barrier.
template <int KEEP>
__device__ __forceinline__ void ring_barrier() {
  static_assert(KEEP >= 0 && KEEP <= 63, "vector-memory counter range");
  // s_waitcnt vmcnt(KEEP) expcnt(7) lgkmcnt(0): vmcnt bits [3:0] and [15:14]
  constexpr int imm = (KEEP & 15) | ((KEEP >> 4) << 14) | (7 << 4);
  __builtin_amdgcn_s_waitcnt(imm);
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Pairs of scheduling groups, N times: S1 instructions of class M1, then S2 of class M2
// (classes as in __builtin_amdgcn_sched_group_barrier: 0x008 matrix core, 0x010 vector
// memory, 0x100 LDS read).
template <int N, int M1, int S1, int M2, int S2>
__device__ __forceinline__ void sched_pairs() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(M1, S1, 0);
    __builtin_amdgcn_sched_group_barrier(M2, S2, 0);
    sched_pairs<N - 1, M1, S1, M2, S2>();
  }
}

}  // namespace lrs
