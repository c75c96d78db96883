// FP64 and int reductions over aligned groups of 2^LG lanes of a wave64, used
// by the three- and n-dimensional kernels (their bounds are doubles).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rgbd {

// Cross-lane moves within aligned groups: quad_perm xor 1 and xor 2, row
// half-mirror (8), row mirror (16) as DPP; the swizzle swap of 16 (32) and
// the other half of the wave (64).  A double moves as its two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)dpp_i<CTRL>((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)dpp_i<CTRL>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double swz16_d(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)u, 0x401F);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), 0x401F);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int imin_(int a, int b) { return a < b ? a : b; }

// IEEE minNum as one instruction: the operands are results of arithmetic
// or copies of them (never signalling NaNs), so the quieting the compiler
// adds around fmin is not needed; a quiet NaN operand (from an invalid row,
// whose LP is reported INVALID) is dropped.
__device__ __forceinline__ double vmin_d(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Smallest value over the group (every lane gets it), and the smallest int.
template <int LG>
__device__ __forceinline__ double group_min_d(double v) {
    if (LG >= 1) v = vmin_d(v, dpp_d<0xB1>(v));
    if (LG >= 2) v = vmin_d(v, dpp_d<0x4E>(v));
    if (LG >= 3) v = vmin_d(v, dpp_d<0x141>(v));
    if (LG >= 4) v = vmin_d(v, dpp_d<0x140>(v));
    if (LG >= 5) v = vmin_d(v, swz16_d(v));
    if (LG >= 6) v = vmin_d(v, __shfl_xor(v, 32));
    return v;
}
template <int LG>
__device__ __forceinline__ int group_min_i(int v) {
    if (LG >= 1) v = imin_(v, dpp_i<0xB1>(v));
    if (LG >= 2) v = imin_(v, dpp_i<0x4E>(v));
    if (LG >= 3) v = imin_(v, dpp_i<0x141>(v));
    if (LG >= 4) v = imin_(v, dpp_i<0x140>(v));
    if (LG >= 5) v = imin_(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));
    if (LG >= 6) v = imin_(v, __shfl_xor(v, 32));
    return v;
}

}  // namespace rgbd
