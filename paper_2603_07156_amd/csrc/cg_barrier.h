// cg_barrier.h -- the grid-wide barrier of the cooperative CG kernels (cg_persistent.hip,
// cg_pipe.hip) on gfx950.
//
// An arrival counter, zeroed before the launch and never reset: barrier k returns once the
// counter reaches k * grid.  Every wave waits for its own stores, then one wave per
// workgroup releases them at device scope (the L2 of each XCD is written back) before
// arriving, and acquires after the wait, so the phase's writes of every workgroup are seen
// by every other.  The wait is bounded: a workgroup that waits longer than BAR_SPIN polls
// raises the error flag (bar[1]) and leaves, so a fault in the barrier ends the kernel with
// an error instead of a hang.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace ibsn {

constexpr int64_t BAR_SPIN = 1ll << 22;   // polls (each after s_sleep) before giving up

// Grid-wide barrier number `target / grid`; false (every thread) when it timed out or
// another workgroup raised the error flag.  A workgroup barrier alone does not wait for
// the other waves' stores, hence the wait in every wave first.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned target, int *sflag)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        // one release per workgroup: writes the L2's dirty lines back for the other XCDs
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int64_t k = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                ++k > BAR_SPIN) {
                ok = 0;
                __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        // one acquire per workgroup: invalidates this CU's L1 and stale L2 lines
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *sflag = ok;
    }
    __syncthreads();
    return *sflag != 0;
}

}  // namespace ibsn
