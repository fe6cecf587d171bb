// gde_device.h -- device helpers shared by the plain and batched kernels:
// wavefront scans and workgroup-aggregated reservations on shared counters.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gde_internal.h"

namespace gde {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }
__device__ __forceinline__ unsigned long long lanemask_lt() { return (1ull << lane()) - 1ull; }

__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(v, off);
        if (lane() >= off) v += y;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_incl_scan64(unsigned long long v) {
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        unsigned long long y = __shfl_up(v, off);
        if (lane() >= off) v += y;
    }
    return v;
}

// Workgroup-aggregated reservation: every thread asks for c slots; the
// workgroup adds its total to *counter with ONE atomic and each thread gets the
// start of its own slots (thread order inside the workgroup).  All threads of
// the workgroup must call it.
__device__ __forceinline__ int block_reserve(int c, int32_t *counter) {
    __shared__ int s_w[kMaxWaves];
    __shared__ int s_base;
    const int incl = wave_incl_scan(c);
    const int wid = threadIdx.x / kWave;
    if (lane() == kWave - 1) s_w[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
            const int v = s_w[i];
            s_w[i] = tot;
            tot += v;
        }
        s_base = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    const int r = s_base + s_w[wid] + incl - c;
    __syncthreads();  // the shared slots are reused by the next call
    return r;
}

// The same for a packed pair (count << 32 | amount); no carry crosses bit 32.
__device__ __forceinline__ unsigned long long block_reserve64(unsigned long long c, unsigned long long *counter) {
    __shared__ unsigned long long s_w64[kMaxWaves];
    __shared__ unsigned long long s_base64;
    const unsigned long long incl = wave_incl_scan64(c);
    const int wid = threadIdx.x / kWave;
    if (lane() == kWave - 1) s_w64[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0ull;
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
            const unsigned long long v = s_w64[i];
            s_w64[i] = tot;
            tot += v;
        }
        s_base64 = tot ? atomicAdd(counter, tot) : 0ull;
    }
    __syncthreads();
    const unsigned long long r = s_base64 + s_w64[wid] + incl - c;
    __syncthreads();
    return r;
}

}  // namespace gde
