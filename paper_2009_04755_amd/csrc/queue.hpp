// Device side of the work queue that persistent kernels pull tiles from.
//
// Section IV-B balances load with work stealing: idle workers take tasks from other
// workers, the largest first, and prefer their own node.  On one GPU each persistent
// workgroup pops the next item of its own XCD's segment (hardware dispatches
// workgroup b to XCD b mod 8, so the segment's items share that XCD's L2); when the
// segment is drained it steals from the other segments in turn.  Items are ordered
// by the host planner (largest first where costs differ).  A pop is one relaxed
// check plus one atomicAdd on the segment's counter; counters sit on separate
// 128-byte lines.
#pragma once

#include "common.hpp"

namespace rk {

__device__ __forceinline__ int queue_pop(const QueueArgs &q)
{
    const int nseg = q.nseg;
    const int home = (int)(blockIdx.x % (unsigned)nseg);
    for (int s = 0; s < nseg; ++s) {
        int g = home + s;
        if (g >= nseg) g -= nseg;
        const int b = q.seg[g], len = q.seg[g + 1] - b;
        int *h = q.heads + g * HEAD_STRIDE;
        if (__hip_atomic_load(h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= len) continue;
        const int k = atomicAdd(h, 1);
        if (k < len) {
            if (q.ledger) atomicAdd(q.ledger + b + k, 1);
            return b + k;
        }
    }
    return -1;
}

// Pop by thread 0, broadcast to the workgroup through LDS.  The caller's loop body
// must contain at least one __syncthreads() between consecutive calls.  `prev` is thread
// 0's previous item (-1 before the first call): with a trace, the wall clock before the
// pop ends the previous item and the clock after it starts the new one, and the new item
// records its workgroup (the per-tile timeline of Section IV-C's profiling).
__device__ __forceinline__ int queue_pop_wg(const QueueArgs &q, int *slot, int &prev)
{
    if (threadIdx.x == 0) {
        if (q.trace && prev >= 0) q.trace[3 * (int64_t)prev + 1] = wall_clock64();
        const int it = queue_pop(q);
        if (q.trace && it >= 0) {
            q.trace[3 * (int64_t)it] = wall_clock64();
            q.trace[3 * (int64_t)it + 2] = blockIdx.x;
        }
        prev = it;
        *slot = it;
    }
    __syncthreads();
    return *slot;
}

}  // namespace rk
