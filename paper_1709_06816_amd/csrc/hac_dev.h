// Device helpers shared by the merge engines (hac_engine.hip, hac_rounds.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Wave-wide reductions from the ROCm device library (DPP lane moves, no LDS
// round trips); the result is uniform across the wave.  Call with every lane
// of the wave active.
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_min_u64(unsigned long long);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);

__device__ __forceinline__ uint64_t wave_min(uint64_t v) { return __ockl_wfred_min_u64(v); }
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) { return __ockl_wfred_add_u64(v); }

}  // namespace hac
