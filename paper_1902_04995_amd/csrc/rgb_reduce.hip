// Segment-minimum microbenchmark: the reduction step of a 1D LP's work units
// (Sec. 3) done four ways, over segments of `c` consecutive values (c = the
// number of work units meeting in one bound, the contention).
//
//   LDS_ATOMIC   every value does an LDS min on its segment's slot
//                (the paper's shared-memory atomics), then one lane per
//                segment writes the slot out;
//   GLOBAL_ATOMIC every value does a device-memory min on its output slot;
//   DPP          butterfly over aligned lane groups (quad permutes, row
//                mirrors, a swizzle, a cross-half shuffle: what the group
//                kernel uses); segments longer than a wave finish with LDS
//                atomics across the block's waves;
//   SERIAL       one lane walks its whole segment (no cross-lane step).
//
// Floats are compared through order-preserving integer keys, so every method
// returns the exact minimum.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rgb.h"

namespace {

__device__ __forceinline__ int key_of(float f) {
    int k = __builtin_bit_cast(int, f);
    return k ^ ((k >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float float_of(int k) { return __builtin_bit_cast(float, k ^ ((k >> 31) & 0x7fffffff)); }

constexpr int kBlock = 256;

// LDS slots of one block: kBlock / c segments when c <= kBlock, else one
// partial segment (c is a power of two, so blocks never straddle segments).
__global__ __launch_bounds__(kBlock) void k_lds_atomic(const float* in, float* out, int64_t n, int c) {
    __shared__ int slot[kBlock];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kBlock + t;
    slot[t] = 0x7fffffff;
    __syncthreads();
    const int seg_in_block = c >= kBlock ? 0 : t / c;
    if (i < n) atomicMin(&slot[seg_in_block], key_of(in[i]));
    __syncthreads();
    if (c >= kBlock) {
        if (t == 0 && i < n) atomicMin(reinterpret_cast<int*>(out) + i / c, slot[0]);  // out pre-filled with +max keys
    } else if (t % c == 0 && i < n) {
        out[i / c] = float_of(slot[seg_in_block]);
    }
}

__global__ __launch_bounds__(kBlock) void k_global_atomic(const float* in, int* out_keys, int64_t n, int c) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) atomicMin(out_keys + i / c, key_of(in[i]));
}

template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

__global__ __launch_bounds__(kBlock) void k_dpp(const float* in, float* out, int* out_keys, int64_t n, int c) {
    __shared__ int slot[kBlock / 64];  // one per segment of the block when 64 < c <= kBlock, else slot 0
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kBlock + t;
    if (t < kBlock / 64) slot[t] = 0x7fffffff;
    int v = i < n ? key_of(in[i]) : 0x7fffffff;
    const int w = c < 64 ? c : 64;
    if (w >= 2) v = imin(v, dpp<0xB1>(v));
    if (w >= 4) v = imin(v, dpp<0x4E>(v));
    if (w >= 8) v = imin(v, dpp<0x141>(v));
    if (w >= 16) v = imin(v, dpp<0x140>(v));
    if (w >= 32) v = imin(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));
    if (w >= 64) v = imin(v, __shfl_xor(v, 32));
    if (c <= 64) {
        if ((t & (c - 1)) == 0 && i < n) out[i / c] = float_of(v);
        return;
    }
    const int seg_in_block = c >= kBlock ? 0 : t / c;
    __syncthreads();
    if ((t & 63) == 0) atomicMin(&slot[seg_in_block], v);
    __syncthreads();
    if (c <= kBlock) {
        if (t % c == 0 && i < n) out[i / c] = float_of(slot[seg_in_block]);
    } else if (t == 0 && i < n) {
        atomicMin(out_keys + i / c, slot[0]);
    }
}

__global__ __launch_bounds__(kBlock) void k_serial(const float* in, float* out, int64_t n, int c) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t lo = s * c;
    if (lo >= n) return;
    int best = 0x7fffffff;
    for (int64_t i = lo; i < lo + c && i < n; ++i) best = imin(best, key_of(in[i]));
    out[s] = float_of(best);
}

__global__ void k_fill_keys(int* keys, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = 0x7fffffff;
}

__global__ void k_keys_to_float(int* keys, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) reinterpret_cast<float*>(keys)[i] = float_of(keys[i]);
}

}  // namespace

extern "C" rgb_err_t rgb_reduce_bench_run(int32_t method, int32_t contention, int64_t n, const float* in, float* out,
                                          void* stream) {
    if (n < 0 || (n > 0 && (!in || !out))) return RGB_ERR_INVALID_ARG;
    if (contention < 2 || contention > 4096 || (contention & (contention - 1)) != 0) return RGB_ERR_INVALID_ARG;
    if (n % contention != 0) return RGB_ERR_INVALID_ARG;
    if (n == 0) return RGB_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int c = contention;
    const int64_t segs = n / c;
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    const unsigned seg_blocks = (unsigned)((segs + kBlock - 1) / kBlock);
    int* keys = reinterpret_cast<int*>(out);
    switch (method) {
        case RGB_REDUCE_LDS_ATOMIC:
            if (c >= kBlock) hipLaunchKernelGGL(k_fill_keys, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(kBlock), 0, st, in, out, n, c);
            if (c >= kBlock) hipLaunchKernelGGL(k_keys_to_float, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            break;
        case RGB_REDUCE_GLOBAL_ATOMIC:
            hipLaunchKernelGGL(k_fill_keys, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            hipLaunchKernelGGL(k_global_atomic, dim3(blocks), dim3(kBlock), 0, st, in, keys, n, c);
            hipLaunchKernelGGL(k_keys_to_float, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            break;
        case RGB_REDUCE_DPP:
            if (c > kBlock) hipLaunchKernelGGL(k_fill_keys, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            hipLaunchKernelGGL(k_dpp, dim3(blocks), dim3(kBlock), 0, st, in, out, keys, n, c);
            if (c > kBlock) hipLaunchKernelGGL(k_keys_to_float, dim3(seg_blocks), dim3(kBlock), 0, st, keys, segs);
            break;
        case RGB_REDUCE_SERIAL:
            hipLaunchKernelGGL(k_serial, dim3(seg_blocks), dim3(kBlock), 0, st, in, out, n, c);
            break;
        default:
            return RGB_ERR_INVALID_ARG;
    }
    return hipGetLastError() == hipSuccess ? RGB_OK : RGB_ERR_DEVICE;
}
