// Grid-wide barrier for persistent cooperative kernels (every workgroup
// resident), shared by the device-resident level loops.
//  - Two levels: eight group counters (workgroup b in group b % 8, which is
//    also its XCD under round-robin placement), each on its own cache line,
//    then one top counter and a generation word.
//  - Every wait is bounded: a wait that exceeds its budget sets the failure
//    flag, and every workgroup sees the flag at its next barrier and leaves,
//    so the kernel always finishes.
//  - Stores before the barrier are visible to every workgroup after it: one
//    release fence before arriving, one acquire fence after the wait.
#pragma once

#include "internal.h"

namespace byo {

constexpr int GS_GROUPS = 8;
constexpr int GS_PAD = 32;  // counters 128 bytes apart

struct grid_sync {
  unsigned arrive[GS_GROUPS * GS_PAD];
  unsigned top[GS_PAD];
  unsigned gen[GS_PAD];
  unsigned fail[GS_PAD];
};

// Relaxed agent-scope loads read the coherent copy without cache
// maintenance; the barrier's fences order them (an acquire load in the spin
// loop would invalidate the L2 on every poll).
__device__ __forceinline__ unsigned ld_rlx(unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_rlx64(unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// false if this workgroup gave up waiting or saw the failure flag
__device__ inline bool grid_barrier(grid_sync *c, unsigned nblocks, unsigned spin_limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned grp = blockIdx.x % GS_GROUPS;
    const unsigned gsize = (nblocks - grp + GS_GROUPS - 1) / GS_GROUPS;
    const unsigned ngroups = nblocks < (unsigned)GS_GROUPS ? nblocks : (unsigned)GS_GROUPS;
    const unsigned g = ld_rlx(&c->gen[0]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    bool released = false;
    unsigned a = __hip_atomic_fetch_add(&c->arrive[grp * GS_PAD], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == gsize - 1) {
      __hip_atomic_store(&c->arrive[grp * GS_PAD], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned t = __hip_atomic_fetch_add(&c->top[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t == ngroups - 1) {
        __hip_atomic_store(&c->top[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&c->gen[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        released = true;
      }
    }
    if (!released) {
      unsigned spins = 0;
      while (ld_rlx(&c->gen[0]) == g) {
        if (++spins > spin_limit || ld_rlx(&c->fail[0])) {
          __hip_atomic_store(&c->fail[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ld_rlx(&c->fail[0])) ok = 0;
  }
  __syncthreads();
  return ok != 0;
}

}  // namespace byo
