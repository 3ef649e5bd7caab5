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

// Data-parallel-primitive move of a double within rows of 16 lanes (both
// 32-bit halves with the same control; every lane of the wavefront active).
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ inline double read_lane(double v, int lane) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over each row of 16 lanes (lanes 16r .. 16r + 15), the same value in
// every lane of the row: rotations by 8, 4, 2, 1.  Every lane must be active.
__device__ inline double row16_sum(double v) {
    v += dpp_move<0x128>(v);  // row_ror:8
    v += dpp_move<0x124>(v);  // row_ror:4
    v += dpp_move<0x122>(v);  // row_ror:2
    v += dpp_move<0x121>(v);  // row_ror:1
    return v;
}

// Sum over the wavefront, the same value in every lane, in a fixed order: row
// rotations by 8, 4, 2, 1 give every lane its 16-lane row's sum, then the four
// row sums are added as (r0 + r1) + (r2 + r3).  Every lane must be active.
template <>
__device__ inline double wave_sum<double>(double v) {
    v = row16_sum(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
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
