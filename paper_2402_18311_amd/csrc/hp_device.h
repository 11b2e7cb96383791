// Device-side helpers of libhybro: wave/block reductions and fixed-point conversions.
#pragma once
#include "hp_internal.h"

namespace hp {

__device__ __forceinline__ int64_t q16(double v) { return __double2ll_rn(v * 65536.0); }
__device__ __forceinline__ int64_t q12(double v) { return __double2ll_rn(v * 4096.0); }

template <typename T> __device__ __forceinline__ T dev_exp(T v);
template <> __device__ __forceinline__ float dev_exp<float>(float v) { return expf(v); }
template <> __device__ __forceinline__ double dev_exp<double>(double v) { return exp(v); }

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __int_as_float(0x7f800000); }
template <> __device__ __forceinline__ double pos_inf<double>() {
    return __longlong_as_double(0x7ff0000000000000LL);
}

// Reductions inside aligned groups of G lanes (G a power of two <= 64); every lane of the
// group gets the result.  The xor butterfly is a fixed order, so results are reproducible.
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_max(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, G));
    return v;
}
template <int G, typename T> __device__ __forceinline__ T group_min(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, G));
    return v;
}

// Block-wide reductions for kBlock = 256 threads (4 waves); all threads get the result.
// `red` is a __shared__ scratch of >= 4 elements; the leading barrier makes reuse safe.
template <typename T> __device__ __forceinline__ T block_sum(T v, T *red) {
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}
template <typename T> __device__ __forceinline__ T block_max(T v, T *red) {
    v = group_max<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return max(max(red[0], red[1]), max(red[2], red[3]));
}
template <typename T> __device__ __forceinline__ T block_min(T v, T *red) {
    v = group_min<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return min(min(red[0], red[1]), min(red[2], red[3]));
}

// Map a block index inside a bucket of nb blocks (nb a multiple of kXcds) so that each XCD
// (which receives blocks i with i % 8 == xcd) works on one contiguous eighth of the bucket.
__device__ __forceinline__ int xcd_remap(int i, int nb) {
    const int q = nb / kXcds;
    return (i % kXcds) * q + i / kXcds;
}

}  // namespace hp
