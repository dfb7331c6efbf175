// rom_common.h -- device helpers shared by the gfx950 kernels of librom.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "rom_device.h"
#include "rom_kernels.h"

namespace rom {

// ------------------------------------------------------------------------------------ helpers
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform64(int64_t x)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
    return ((int64_t)hi << 32) | (unsigned)lo;
}

// Strip-edge hand-off between wavefronts that may sit on different XCDs.  The edge words
// themselves are written and read with device-scope (agent) relaxed atomic accesses, which the
// hardware keeps coherent across the per-XCD L2 caches word by word; the producer then waits for
// its stores to complete (s_waitcnt vmcnt(0)) before it publishes the progress counter.  This
// avoids the whole-L2 write-back / invalidate that a release / acquire fence pair costs.
template <typename T>
__device__ __forceinline__ void edge_store(T* p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ T edge_load(const T* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ __forceinline__ void stores_complete() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Sweep duration on the device real-time clock, taken from the persistent workgroups' ticket
// claims instead of an atomic per workgroup (hundreds of same-address device-scope atomics at a
// launch's start and end serialize: c5 and c3 steps ran 3 % and 6 % slower with them).  The first
// claim (ticket 0) marks the start; every workgroup ends with one failing claim after its last
// task, so claim ntickets + gridDim.x - 1 comes after all work and marks the end.  Plain stores:
// each value has one writer, and the combine step reads them after this kernel.
__device__ __forceinline__ void sweep_clock(Ctl* ctl, int claim, int ntickets)
{
    if (claim == 0) ctl->t_first = wall_clock64();
    else if (claim == ntickets + (int)gridDim.x - 1) ctl->t_last = wall_clock64();
}

// Bounded waits.  A wait gives up and records ctl->error after `limit` polls or after `ticks`
// ticks of the device real-time clock (wall_clock64), whichever comes first, and leaves early
// without recording anything once another wave has recorded an error (checked every 64 polls).
// The clock bound keeps a timed-out wait short however long a contended device-scope poll takes
// (a poll count alone bounds it only by polls x poll latency), so every wave exits and the host
// reports ROM_E_DEVICE.  Returns true when the wait gave up.
__device__ __forceinline__ bool wait_gave_up(int spins, unsigned long long t0, Ctl* ctl, int limit, long long ticks)
{
    if (spins >= limit) {
        __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    }
    if ((spins & 63) == 0) {
        if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return true;
        if ((long long)(wall_clock64() - t0) > ticks) {
            __hip_atomic_store(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return true;
        }
    }
    return false;
}

// Wait until *p >= target (the strip below has finished chunk c of this epoch).
__device__ __forceinline__ void wait_progress(long long* p, long long target, Ctl* ctl, int limit, long long ticks)
{
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        const unsigned long long t0 = wall_clock64();
        int spins = 0;
        while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wait_gave_up(++spins, t0, ctl, limit, ticks)) break;
        }
    }
    asm volatile("" ::: "memory");  // edge loads stay after the poll
}

// Wait until an LDS counter of the workgroup reaches `target` (bounded like wait_progress).
__device__ __forceinline__ void lds_wait(int* p, int target, Ctl* ctl, int limit, long long ticks)
{
    if (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
        const unsigned long long t0 = wall_clock64();
        int spins = 0;
        while (__hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (wait_gave_up(++spins, t0, ctl, limit, ticks)) break;
        }
    }
}

template <typename T>
__device__ __forceinline__ T to_T(double x) { return (T)x; }

#ifndef ROM_ROW_UNROLL
#define ROM_ROW_UNROLL 0
#endif


}  // namespace rom
