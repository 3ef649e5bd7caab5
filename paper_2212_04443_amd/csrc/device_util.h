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

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC 2011): ten rounds of
// (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2, c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
// with the key bumped by the Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)M0 * c[0];
        const uint64_t p1 = (uint64_t)M1 * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
}

}  // namespace chebdav
