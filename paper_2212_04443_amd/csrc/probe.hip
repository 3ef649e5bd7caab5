// Measurement utility: gathers of whole rows at uniformly random positions of a
// row-major table, with the sparse step's load shape (G lanes per row, 16 bytes
// per lane, 16 rows in flight per group).  On a graph without locality whose
// gathered block exceeds the caches (Table 2's skewed matrices, the Chung-Lu
// stand-in) the sparse step is a sequence of such gathers, one per nonzero, so
// the time of nnz of them bounds the step from below on the GPU it runs on.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kProbeBlocks = 2048, kProbeThreads = 256, kProbeBatch = 16;

// SplitMix64 finalizer (Steele, Lea and Flood, 2014): a well-mixed 64-bit value per
// (group, draw), reduced to a row index by a 64 x 64 -> high 64-bit product.
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <int G>
__global__ void __launch_bounds__(kProbeThreads) k_probe_gather(const double2 *__restrict__ table, int64_t rows,
                                                                int64_t per_group, uint64_t seed,
                                                                double *__restrict__ out) {
    constexpr int GPB = kProbeThreads / G;
    const int64_t grp = (int64_t)blockIdx.x * GPB + threadIdx.x / G;
    const int gl = threadIdx.x & (G - 1);
    double acc = 0.0;
    for (int64_t i = 0; i < per_group; i += kProbeBatch) {
        double2 v[kProbeBatch];
#pragma unroll
        for (int u = 0; u < kProbeBatch; ++u) {
            const uint64_t h = mix64(seed ^ ((uint64_t)grp << 24) ^ (uint64_t)(i + u));
            const int64_t r = (int64_t)__umul64hi(h, (uint64_t)rows);  // < rows
            v[u] = (i + u < per_group) ? table[r * G + gl] : double2{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < kProbeBatch; ++u) acc += v[u].x + v[u].y;
    }
    // one value per group keeps the loads live
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) out[(int64_t)blockIdx.x * (kProbeThreads / kWave) + threadIdx.x / kWave] = acc;
}

}  // namespace

int64_t probe_gather_out_len() { return (int64_t)kProbeBlocks * (kProbeThreads / kWave); }

chebdav_status probe_gather(const void *table, int64_t rows, int row_bytes, int64_t gathers, uint64_t seed,
                            double *out, int64_t *performed, hipStream_t st) {
    if (!table || !out) return fail(CHEBDAV_EINVAL, "table or out is NULL");
    if (rows < 1 || gathers < 0) return fail(CHEBDAV_EINVAL, "need rows >= 1 and gathers >= 0");
    if (reinterpret_cast<uintptr_t>(table) % 16) return fail(CHEBDAV_EINVAL, "table must be 16-byte aligned");
    if (row_bytes != 128 && row_bytes != 256 && row_bytes != 512)
        return fail(CHEBDAV_EINVAL, "row_bytes must be 128, 256 or 512");
    const auto *t = static_cast<const double2 *>(table);
    const int64_t groups = (int64_t)kProbeBlocks * (kProbeThreads / (row_bytes / 16));
    const int64_t per_group = gathers == 0 ? 0 : (gathers + groups - 1) / groups;
    if (performed) *performed = per_group * groups;
    switch (row_bytes) {
        case 128:
            hipLaunchKernelGGL(k_probe_gather<8>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, t, rows, per_group, seed, out);
            break;
        case 256:
            hipLaunchKernelGGL(k_probe_gather<16>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, t, rows, per_group, seed, out);
            break;
        case 512:
            hipLaunchKernelGGL(k_probe_gather<32>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, t, rows, per_group, seed, out);
            break;
        default:
            return fail(CHEBDAV_EINVAL, "row_bytes must be 128, 256 or 512");  // checked above
    }
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
