// Device-side helpers: wave/block scans and reductions (64-wide wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chebdav {

constexpr int kWave = 64;

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

template <typename T>
__device__ inline T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive scan over the block (blockDim.x a multiple of 64, <= 1024).
// `total` receives the block sum.  Contains __syncthreads(): call from all threads.
template <typename T>
__device__ inline T block_excl_scan(T v, T *total) {
    __shared__ T wsum[16];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
    for (int i = 0; i < nw; ++i) {
        T s = wsum[i];
        if (i < w) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Sum over the block, result valid in every thread.  Contains __syncthreads().
template <typename T>
__device__ inline T block_sum(T v) {
    __shared__ T wsum[16];
    const int lane = lane_id();
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    v = wave_sum(v);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    T all = 0;
    for (int i = 0; i < nw; ++i) all += wsum[i];
    __syncthreads();
    return all;
}

}  // namespace chebdav
