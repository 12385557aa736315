// micx_device.h -- device helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "micx_internal.h"

namespace micx {

__device__ __forceinline__ int64_t tri_offset(int64_t i, int64_t m) {
    return i * m - i * (i + 1) / 2;
}

// Pair (i, j) of batch-local pair index pl: an explicit list, or the
// row-major upper triangle of an m-variable matrix from global index p0.
__device__ __forceinline__ void pair_of(const PairSource &ps, int pl, int &i, int &j) {
    if (ps.pairs) {
        i = ps.pairs[2 * pl];
        j = ps.pairs[2 * pl + 1];
        return;
    }
    const int64_t P = ps.p0 + pl, m = ps.m;
    const double mm = 2.0 * (double)m - 1.0;
    int64_t a = (int64_t)floor((mm - sqrt(mm * mm - 8.0 * (double)P)) * 0.5);
    if (a < 0) a = 0;
    if (a > m - 2) a = m - 2;
    while (a + 1 <= m - 2 && tri_offset(a + 1, m) <= P) a++;
    while (a > 0 && tri_offset(a, m) > P) a--;
    i = (int)a;
    j = (int)(P - tri_offset(a, m) + a + 1);
}

// Orders this wavefront's LDS accesses (writes before the sync are visible to
// reads after it); waves of a workgroup run independently between the calls.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Completes this wavefront's global stores before its later global loads.
__device__ __forceinline__ void global_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

}  // namespace micx
