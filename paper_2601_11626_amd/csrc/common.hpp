// Shared device/host helpers for the cmsvd HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <utility>

#define CMSVD_WAVE 64

namespace cmsvd {

// Raises a kernel's dynamic-LDS limit to `bytes`, once per function and device: the
// attribute persists, so launches recorded into a graph capture find it already set and
// make no runtime call besides the launch.
inline void lds_limit(const void* fn, int bytes) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    int& cur = done[{fn, dev}];
    if (cur >= bytes) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess) cur = bytes;
    else (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wave / block reductions (deterministic: fixed butterfly order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    return __shfl_xor(v, mask, CMSVD_WAVE);
}

// Cross-lane moves that stay on the VALU (no LDS round trip): DPP within rows of
// 16 lanes and the gfx950 permlane16/32 swaps across rows.  Lane semantics were
// checked on the device: quad_perm 0xB1 = lane^1, 0x4E = lane^2, row_half_mirror
// pairs the two quads of every 8-lane group, row_ror:8 = lane^8 within 16 lanes.
// Every control used here reads a valid lane, so the moves need no "old" operand.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Pairwise reductions through the swaps: lanes 0..31 receive x(l) + x(l^32) and
// lanes 32..63 receive y(l) + y(l^32); with x == y this is the sum over lane^32.
__device__ __forceinline__ double add_swap32(double x, double y) {
    const auto a = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    const auto b = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
// Rows of 16 lanes: even rows receive x(l) + x(l^16), odd rows y(l) + y(l^16).
__device__ __forceinline__ double add_swap16(double x, double y) {
    const auto a = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false, false);
    const auto b = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
__device__ __forceinline__ double add_swap32(double v) { return add_swap32(v, v); }
__device__ __forceinline__ double add_swap16(double v) { return add_swap16(v, v); }

// Sum over each group of 8 consecutive lanes (every lane of the group gets it).
__device__ __forceinline__ double sum_lanes8(double v) {
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    return v;
}

// Sum over the 8 lanes sharing lane % 8 (every lane of the set gets it).
__device__ __forceinline__ double sum_stride8(double v) {
    v += dpp_move<0x128>(v);
    v = add_swap16(v);
    return add_swap32(v);
}

__device__ __forceinline__ double wave_sum(double v) { return sum_stride8(sum_lanes8(v)); }

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
