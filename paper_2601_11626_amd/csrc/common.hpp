// Shared device/host helpers for the cmsvd HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CMSVD_WAVE 64

namespace cmsvd {

// ---------------------------------------------------------------------------
// Wave / block reductions (deterministic: fixed butterfly order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, CMSVD_WAVE);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += shfl_xor_d(v, o);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, shfl_xor_d(v, o));
    return v;
}

// Sum over the whole block; every thread receives the result.  `red` must hold
// blockDim.x / 64 doubles of LDS.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ double block_max(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    return s;
}

// Error-free transformation a + b = s + e (Knuth TwoSum).
__device__ __host__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Double-double accumulator (hi, lo) += x.
__device__ __host__ __forceinline__ void dd_add(double& hi, double& lo, double x) {
    double s, e;
    two_sum(hi, x, s, e);
    lo += e;
    hi = s;
}

template <typename T>
__device__ __forceinline__ double to_d(T x) {
    return static_cast<double>(x);
}

}  // namespace cmsvd
