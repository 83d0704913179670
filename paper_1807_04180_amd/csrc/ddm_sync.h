// Device-side meeting helpers shared by the substitution kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ddm {

// Meetings of workgroups without cache maintenance: an agent-scope fence on
// this chip writes back and invalidates the whole L2 (at one exchange per
// block and 256 workgroups that costs more than the block itself; at the one
// meeting per launch of the two chains of a subdomain it cost 0.19 ms of a
// 2.46 ms split local solve).  The exchanged words and the flags are instead
// relaxed agent-scope atomics (coherent at the agent level without touching
// other cached data); the writer waits for its stores to complete (s_waitcnt
// 0: stores count in vmcnt here) before a barrier and the flag store, and
// the reader loads the words only after it has seen the flag (and a
// barrier).  Every wait is bounded (spin_limit) and stops at once after a
// sticky abort.
__device__ inline void wait_flag_relaxed(int *f, int target, int *abort_flag, int spin_limit) {
    if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins >= spin_limit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
}

__device__ inline void xstore(double2 *p, double2 v) {
    unsigned long long *q = (unsigned long long *)p;
    __hip_atomic_store(q, __double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, __double_as_longlong(v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void xstore(float2 *p, float2 v) {
    const unsigned long long w = (unsigned long long)__float_as_uint(v.x) |
                                 ((unsigned long long)__float_as_uint(v.y) << 32);
    __hip_atomic_store((unsigned long long *)p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double2 xload(double2 *p) {
    unsigned long long *q = (unsigned long long *)p;
    return make_double2(__longlong_as_double(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
                        __longlong_as_double(__hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ inline float2 xload(float2 *p) {
    const unsigned long long w =
        __hip_atomic_load((unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((unsigned)w), __uint_as_float((unsigned)(w >> 32)));
}

// one component (real or imaginary part) of a complex value, stored the same
// way (read back whole with xload)
__device__ inline void xstore_r(float *p, float v) {
    __hip_atomic_store((unsigned *)p, __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void xstore_r(double *p, double v) {
    __hip_atomic_store((unsigned long long *)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ddm
