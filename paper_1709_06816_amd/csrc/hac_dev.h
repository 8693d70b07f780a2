// Device helpers shared by the merge engines (hac_engine.hip, hac_rounds.hip,
// hac_scan.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hac.h"

namespace hac {

// Order-preserving map of fp32 onto u32 (zeros are canonical +0 here).
__device__ __forceinline__ uint32_t ord32(float x) {
    uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Table 1 update, fp32, fixed order, no contraction.  Coefficients are fp64
// quotients rounded once to fp32 (ai, aj, bij: the per-merge coefficients of
// the group-average and centroid rows).  Single/complete use the exact closed
// forms min/max of the Table 1 rows (1/2, 1/2, 0, -+1/2).
__device__ __forceinline__ float lw_update(int link, float dki, float dkj, float dij, int ni,
                                           int nj, int nk, float ai, float aj, float bij) {
    float v;
    if (link == HAC_SINGLE) {
        v = fminf(dki, dkj);
    } else if (link == HAC_COMPLETE) {
        v = fmaxf(dki, dkj);
    } else if (link == HAC_AVERAGE) {
        v = __fadd_rn(__fmul_rn(ai, dki), __fmul_rn(aj, dkj));
    } else if (link == HAC_WEIGHTED) {
        v = __fadd_rn(__fmul_rn(0.5f, dki), __fmul_rn(0.5f, dkj));
    } else if (link == HAC_CENTROID) {
        v = __fadd_rn(__fadd_rn(__fmul_rn(ai, dki), __fmul_rn(aj, dkj)), __fmul_rn(bij, dij));
    } else {
        double t = (double)(ni + nj + nk);
        float wi = (float)((double)(ni + nk) / t);
        float wj = (float)((double)(nj + nk) / t);
        float wb = (float)(-(double)nk / t);
        v = __fadd_rn(__fadd_rn(__fmul_rn(wi, dki), __fmul_rn(wj, dkj)), __fmul_rn(wb, dij));
    }
    return v == 0.0f ? 0.0f : v;
}

// Workgroup barrier after which the global stores of every wave of the
// workgroup are complete (acknowledged by this XCD's L2).
//
// Publishing to other workgroups works like this: thread 0 issues an
// agent-scope release fence and then stores a flag or counter; a reader that
// sees it takes an agent-scope acquire.  On gfx950 the release is "write
// back this XCD's L2, then wait for my own wave's memory operations", and a
// plain workgroup barrier waits for no global store at all (each wave counts
// its own stores, and a workgroup-scope release needs no such wait when all
// waves share one CU).  So a store issued by another wave just before the
// barrier can still be in flight when thread 0 writes back the L2 and
// publishes: it then lands in the L2 as a dirty line after the write back,
// and a reader on another XCD, whose acquire only invalidates its own caches,
// fetches the old value from memory.  Making every wave wait for its own
// stores first closes that window: after this barrier, thread 0's release
// covers the writes of the whole workgroup.
__device__ __forceinline__ void barrier_stores_done() {
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt(0) expcnt(0) lgkmcnt(0): this wave's stores are acknowledged
    __syncthreads();
}

// Release before publishing with a relaxed store or atomic (one thread, after
// barrier_stores_done): write this XCD's L2 back, then wait for that write
// back to finish.  The fence alone is not enough here: the compiler places
// the wait that completes the write back (buffer_wbl2) only while the wave
// has other memory operations outstanding, and right after
// barrier_stores_done it has none, so the flag could leave before the data it
// publishes has reached memory and a reader on another XCD would fetch the
// old values.  The explicit wait restores the documented release sequence.
__device__ __forceinline__ void release_agent() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
}
__device__ __forceinline__ void release_system() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __builtin_amdgcn_s_waitcnt(0);
}

// Wave-wide reductions from the ROCm device library (DPP lane moves, no LDS
// round trips); the result is uniform across the wave.  Call with every lane
// of the wave active.
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_min_u64(unsigned long long);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);

__device__ __forceinline__ uint64_t wave_min(uint64_t v) { return __ockl_wfred_min_u64(v); }
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) { return __ockl_wfred_add_u64(v); }


// Grid barrier of a cooperative launch of G workgroups: every workgroup's
// writes before it are visible to every workgroup after it (stores complete,
// then an agent-scope release, a monotonic arrival counter *bar, an
// agent-scope acquire).  `gen` counts this workgroup's barriers.  Returns
// false, the same for every thread of the workgroup, if *abort is raised or
// the wait exceeds `timeout` wall-clock ticks (then *error gets `err_bit`
// and *abort is raised for all).  `stall`: this workgroup does not arrive
// (failure tests), so the others' waits expire.
__device__ inline bool grid_sync(uint32_t *bar, uint32_t *abort, uint32_t *error, uint32_t err_bit, uint32_t &gen,
                                 uint32_t G, uint64_t timeout, bool stall = false) {
    __shared__ uint32_t s_sync_fail;
    barrier_stores_done();
    if (threadIdx.x == 0) {
        ++gen;
        release_agent();
        if (!stall) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = gen * G;
        uint32_t fail = 0;
        const uint64_t t0 = wall_clock64();
        for (uint32_t it = 1;; ++it) {
            if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if ((it & 63u) == 0) {
                if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    fail = 1;
                    break;
                }
                if (wall_clock64() - t0 > timeout) {
                    atomicOr(error, err_bit);
                    __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    fail = 1;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_sync_fail = fail;
    }
    __syncthreads();
    return s_sync_fail == 0;
}

}  // namespace hac
