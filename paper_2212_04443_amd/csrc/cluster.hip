// Clustering tail of spectral clustering (Alg. 1, steps 3 and 4): every row of
// the n x k eigenvector block is scaled to unit length (a zero row stays zero)
// and the rows are grouped by Lloyd's K-means.
//
// Readings: K centres start by farthest-first traversal (Gonzalez, 1985) from
// row floor(u n), u the Philox4x32-10 draw of counter (0, 0, 0, 1) under the
// seed (integer arithmetic); each next centre is the row farthest from its
// nearest chosen centre, ties to the lower row index.  A row joins the nearest
// centre (ties to the lower centre index); a centre moves to the mean of its
// rows and stays put when it has none; rounds stop when no label changes or
// after max_iter rounds.  Squared distances are summed over the coordinates in
// ascending order with separately rounded subtract, multiply and add.
//
// Every floating-point sum over rows is split into fixed row ranges and the
// partial sums are added in a fixed order, so results are deterministic.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kMaxK = 64;        // coordinates per row (columns of the eigenvector block)
constexpr int kMaxClusters = 256;
constexpr int kRowsTpb = 128;    // threads per block of the row kernels
constexpr int kSplits = 1024;    // row ranges of the reductions

// Squared distance; KP >= k is the padded width of the register copy of the row.
// (The products and sums are kept separate: no contraction into fused multiply-add.)
template <int KP>
__device__ inline double sqd(const double (&f)[KP], const double *c, int k) {
#pragma clang fp contract(off)
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        if (j < k) {
            const double t = f[j] - c[j];
            d = d + t * t;
        }
    }
    return d;
}

template <int KP>
__device__ inline void load_row(const double *__restrict__ F, int64_t i, int k, double (&f)[KP]) {
#pragma unroll
    for (int j = 0; j < KP; ++j) f[j] = j < k ? F[i * k + j] : 0.0;
}

// F(i, :) = U(i, :) / ||U(i, :)||_2: one wavefront per row, lanes over columns.
// Every lane forms the sum of squares itself, in ascending coordinate order
// (entries passed lane to lane), then one rounded square root and division.
__global__ void __launch_bounds__(256) k_row_normalize(const double *__restrict__ U, int64_t ldu, int64_t n,
                                                       int k, double *__restrict__ F) {
#pragma clang fp contract(off)
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= n) return;
    const int lane = lane_id();
    const double x = lane < k ? U[r * ldu + lane] : 0.0;
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
        const double xj = __shfl(x, j, kWave);
        s = s + xj * xj;
    }
    const double nr = sqrt(s);
    if (lane < k) F[r * k + lane] = nr > 0.0 ? x / nr : 0.0;
}

// Copy of row `idx` of F into centre slot c (idx read from the device).
__global__ void k_take_row(const double *__restrict__ F, int k, const int64_t *__restrict__ idx, int c,
                           double *__restrict__ C) {
    const int j = threadIdx.x;
    if (j < k) C[(int64_t)c * k + j] = F[idx[0] * k + j];
}

__device__ inline void better(double &bv, int64_t &bi, double v, int64_t i) {
    if (v > bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
    }
}

// Farthest-first step: mind = min(mind, |F_i - C_c|^2) (first == 1: mind = that
// distance), then the block's largest mind with the lowest row index among ties.
template <int KP>
__global__ void __launch_bounds__(kRowsTpb) k_ff_step(const double *__restrict__ F, int64_t n, int k,
                                                      const double *__restrict__ C, int c, int first,
                                                      double *__restrict__ mind, double *__restrict__ bval,
                                                      int64_t *__restrict__ bidx) {
    __shared__ double cs[kMaxK];
    __shared__ double sv[kRowsTpb / kWave];
    __shared__ int64_t si[kRowsTpb / kWave];
    if (threadIdx.x < k) cs[threadIdx.x] = C[(int64_t)c * k + threadIdx.x];
    __syncthreads();
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double f[KP];
        load_row<KP>(F, i, k, f);
        const double d = sqd<KP>(f, cs, k);
        const double m = first ? d : fmin(mind[i], d);
        mind[i] = m;
        better(bv, bi, m, i);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, kWave);
        const int64_t oi = __shfl_xor(bi, o, kWave);
        better(bv, bi, ov, oi);
    }
    if (lane_id() == 0) {
        sv[threadIdx.x / kWave] = bv;
        si[threadIdx.x / kWave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRowsTpb / kWave; ++w) better(bv, bi, sv[w], si[w]);
        bval[blockIdx.x] = bv;
        bidx[blockIdx.x] = bi;
    }
}

// Largest of the per-block maxima (lowest index among ties) -> idx[0].
__global__ void __launch_bounds__(256) k_ff_pick(const double *__restrict__ bval, const int64_t *__restrict__ bidx,
                                                 int nb, int64_t *__restrict__ idx) {
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) better(bv, bi, bval[b], bidx[b]);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, kWave);
        const int64_t oi = __shfl_xor(bi, o, kWave);
        better(bv, bi, ov, oi);
    }
    if (lane_id() == 0) {
        sv[threadIdx.x / kWave] = bv;
        si[threadIdx.x / kWave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) better(bv, bi, sv[w], si[w]);
        idx[0] = bi;
    }
}

// Assignment: label of every row = nearest centre (lower index among ties);
// counts the rows whose label changed (integer atomics).
template <int KP>
__global__ void __launch_bounds__(kRowsTpb) k_assign(const double *__restrict__ F, int64_t n, int k,
                                                     const double *__restrict__ C, int K,
                                                     int32_t *__restrict__ labels, int *__restrict__ changed) {
    extern __shared__ double cs[];  // K x k
    for (int e = threadIdx.x; e < K * k; e += blockDim.x) cs[e] = C[e];
    __syncthreads();
    int ch = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double f[KP];
        load_row<KP>(F, i, k, f);
        double best = sqd<KP>(f, cs, k);
        int bl = 0;
        for (int c = 1; c < K; ++c) {
            const double d = sqd<KP>(f, cs + (int64_t)c * k, k);
            if (d < best) {
                best = d;
                bl = c;
            }
        }
        ch += labels[i] != bl;
        labels[i] = bl;
    }
    ch = wave_sum(ch);
    if (lane_id() == 0 && ch) atomicAdd(changed, ch);
}

// dist[i] = squared distance of row i to the centre it is labelled with.
template <int KP>
__global__ void __launch_bounds__(kRowsTpb) k_label_dist(const double *__restrict__ F, int64_t n, int k,
                                                         const double *__restrict__ C,
                                                         const int32_t *__restrict__ labels,
                                                         double *__restrict__ dist) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double f[KP];
        load_row<KP>(F, i, k, f);
        dist[i] = sqd<KP>(f, C + (int64_t)labels[i] * k, k);
    }
}

// Per row range z: sums of the rows of each cluster (lane j owns coordinate j,
// rows in ascending order) and the row counts.
__global__ void __launch_bounds__(kWave) k_centre_partial(const double *__restrict__ F, int64_t n, int k,
                                                          const int32_t *__restrict__ labels, int K,
                                                          int64_t rows_per_split, double *__restrict__ psum,
                                                          int64_t *__restrict__ pcnt) {
    extern __shared__ double acc[];  // K x k
    int64_t *cnt = reinterpret_cast<int64_t *>(acc + (int64_t)K * k);
    const int j = threadIdx.x;
    for (int e = j; e < K * k; e += kWave) acc[e] = 0.0;
    for (int c = j; c < K; c += kWave) cnt[c] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_split, r1 = min(n, r0 + rows_per_split);
    constexpr int BT = 8;  // rows loaded ahead of their (in-order) accumulation
    for (int64_t rb = r0; rb < r1; rb += BT) {
        int l[BT];
        double x[BT];
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            const int64_t r = rb + t;
            l[t] = r < r1 ? labels[r] : -1;
            x[t] = (r < r1 && j < k) ? F[r * k + j] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < BT; ++t) {
            if (l[t] < 0) break;
            if (j < k) acc[(int64_t)l[t] * k + j] += x[t];
            if (j == 0) cnt[l[t]] += 1;
        }
    }
    __syncthreads();
    double *ps = psum + (int64_t)blockIdx.x * K * k;
    for (int e = j; e < K * k; e += kWave) ps[e] = acc[e];
    for (int c = j; c < K; c += kWave) pcnt[(int64_t)blockIdx.x * K + c] = cnt[c];
}

// C(c, j) = (sum of the split partials) / count; an empty cluster keeps its
// centre.  Thread group zg of a block adds splits zg, zg + 8, ... for 32
// entries; the eight group sums are added in order (fixed order overall).
__global__ void __launch_bounds__(256) k_centre_final(const double *__restrict__ psum,
                                                      const int64_t *__restrict__ pcnt, int S, int K, int k,
                                                      double *__restrict__ C) {
    constexpr int EB = 32, ZG = 8;
    __shared__ double sh[ZG][EB];
    __shared__ int64_t shc[ZG][EB];
    const int el = threadIdx.x % EB, zg = threadIdx.x / EB;
    const int e = blockIdx.x * EB + el;
    const int KK = K * k;
    double sacc = 0.0;
    int64_t m = 0;
    if (e < KK) {
        const int c = e / k;
        for (int z = zg; z < S; z += ZG) {
            sacc += psum[(int64_t)z * KK + e];
            m += pcnt[(int64_t)z * K + c];
        }
    }
    sh[zg][el] = sacc;
    shc[zg][el] = m;
    __syncthreads();
    if (zg == 0 && e < KK) {
        double t = 0.0;
        int64_t mt = 0;
#pragma unroll
        for (int g = 0; g < ZG; ++g) {
            t += sh[g][el];
            mt += shc[g][el];
        }
        if (mt > 0) C[e] = t / (double)mt;
    }
}

// Sum of dist over fixed row ranges, then in order.
__global__ void __launch_bounds__(256) k_sum_partial(const double *__restrict__ x, int64_t n, int64_t rps,
                                                     double *__restrict__ part) {
    const int64_t r0 = (int64_t)blockIdx.x * rps, r1 = min(n, r0 + rps);
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += x[r];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_final(const double *__restrict__ part, int S, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int z = 0; z < S; ++z) s += part[z];
        out[0] = s;
    }
}

__global__ void k_first_index(int64_t n, uint64_t seed, int64_t *__restrict__ idx) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t c[4] = {0u, 0u, 0u, 1u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t u53 = (((uint64_t)c[1] << 32) | c[0]) >> 11;
    // floor(u53 * n / 2^53) with a 128-bit product
    const unsigned __int128 p = (unsigned __int128)u53 * (unsigned __int128)(uint64_t)n;
    idx[0] = (int64_t)(p >> 53);
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t count, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) p[e] = v;
}

struct ClusterWs {
    double *F, *mind, *bval, *psum, *dsum, *out;
    int64_t *bidx, *pcnt, *idx;
    int *changed;
};

int ff_blocks(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(n, kRowsTpb))); }
int splits_for(int64_t n) { return (int)std::min<int64_t>(kSplits, std::max<int64_t>(1, ceil_div(n, 256))); }

ClusterWs cluster_layout(Arena &a, int64_t n, int k, int K) {
    ClusterWs s;
    const int S = splits_for(n), B = ff_blocks(n);
    s.F = a.take<double>((size_t)n * k);
    s.mind = a.take<double>(n);
    s.bval = a.take<double>(B);
    s.bidx = a.take<int64_t>(B);
    s.psum = a.take<double>((size_t)S * K * k);
    s.pcnt = a.take<int64_t>((size_t)S * K);
    s.dsum = a.take<double>(S);
    s.out = a.take<double>(1);
    s.idx = a.take<int64_t>(1);
    s.changed = a.take<int>(1);
    return s;
}

chebdav_status assign(int KP, int B, size_t lds, const double *F, int64_t n, int k, const double *C, int K,
                      int32_t *labels, int *changed, hipStream_t st) {
    switch (KP) {
        case 8: hipLaunchKernelGGL(k_assign<8>, dim3(B), dim3(kRowsTpb), lds, st, F, n, k, C, K, labels, changed); break;
        case 16: hipLaunchKernelGGL(k_assign<16>, dim3(B), dim3(kRowsTpb), lds, st, F, n, k, C, K, labels, changed); break;
        case 32: hipLaunchKernelGGL(k_assign<32>, dim3(B), dim3(kRowsTpb), lds, st, F, n, k, C, K, labels, changed); break;
        default: hipLaunchKernelGGL(k_assign<64>, dim3(B), dim3(kRowsTpb), lds, st, F, n, k, C, K, labels, changed); break;
    }
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace

chebdav_status cluster_ws_bytes(int64_t n, int k, int K, size_t *bytes) {
    if (n < 1 || k < 1 || k > kMaxK || K < 1 || K > kMaxClusters)
        return fail(CHEBDAV_EINVAL, "need n >= 1, 1 <= k <= %d, 1 <= n_clusters <= %d", kMaxK, kMaxClusters);
    Arena a;
    a.counting = true;
    (void)cluster_layout(a, n, k, K);
    *bytes = a.used + 256;
    return CHEBDAV_OK;
}

void *pinned_host(size_t bytes, int slot);

chebdav_status cluster(const double *U, int64_t ldu, int64_t n, int k, int K, int max_iter, uint64_t seed,
                       int32_t *labels, double *centres, int *rounds, double *inertia, void *ws, size_t ws_bytes,
                       hipStream_t st) {
    size_t need = 0;
    CD_TRY(cluster_ws_bytes(n, k, K, &need));
    if (K > n) return fail(CHEBDAV_EINVAL, "n_clusters > n");
    if (ldu < k) return fail(CHEBDAV_EINVAL, "ldu < k");
    if (max_iter < 1) return fail(CHEBDAV_EINVAL, "max_iter must be >= 1");
    if (!U || !labels || !centres) return fail(CHEBDAV_EINVAL, "NULL buffer");
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "cluster workspace too small (%zu < %zu)", ws_bytes, need);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const ClusterWs s = cluster_layout(a, n, k, K);
    int *hchg = static_cast<int *>(pinned_host(2 * sizeof(double), 3));
    if (!hchg) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    const size_t lds_assign = sizeof(double) * (size_t)K * k;
    const size_t lds_partial = sizeof(double) * (size_t)K * k + sizeof(int64_t) * K;
    if (lds_partial > 64 * 1024) return fail(CHEBDAV_EUNSUPPORTED, "n_clusters * (k + 1) must be <= 8192");
    const int KP = k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64;

    // step 3: row normalization
    hipLaunchKernelGGL(k_row_normalize, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, U, ldu, n, k, s.F);
    CD_LAUNCH_CHECK();
    // farthest-first centres
    const int B = ff_blocks(n);
    hipLaunchKernelGGL(k_first_index, dim3(1), dim3(64), 0, st, n, seed, s.idx);
    CD_LAUNCH_CHECK();
    for (int c = 0; c < K; ++c) {
        hipLaunchKernelGGL(k_take_row, dim3(1), dim3(kMaxK), 0, st, s.F, k, s.idx, c, centres);
        CD_LAUNCH_CHECK();
        if (c + 1 == K) break;
        const int first = c == 0 ? 1 : 0;
        switch (KP) {
            case 8: hipLaunchKernelGGL(k_ff_step<8>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, c, first, s.mind, s.bval, s.bidx); break;
            case 16: hipLaunchKernelGGL(k_ff_step<16>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, c, first, s.mind, s.bval, s.bidx); break;
            case 32: hipLaunchKernelGGL(k_ff_step<32>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, c, first, s.mind, s.bval, s.bidx); break;
            default: hipLaunchKernelGGL(k_ff_step<64>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, c, first, s.mind, s.bval, s.bidx); break;
        }
        CD_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ff_pick, dim3(1), dim3(256), 0, st, s.bval, s.bidx, B, s.idx);
        CD_LAUNCH_CHECK();
    }
    // step 4: Lloyd rounds
    const int S = splits_for(n);
    const int64_t rps = ceil_div(n, S);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>(8192, ceil_div(n, 256))), dim3(256), 0, st,
                       labels, n, (int32_t)-1);
    CD_LAUNCH_CHECK();
    int r = 0;
    while (r < max_iter) {
        ++r;
        CD_HIP(hipMemsetAsync(s.changed, 0, sizeof(int), st));
        CD_TRY(assign(KP, B, lds_assign, s.F, n, k, centres, K, labels, s.changed, st));
        hipLaunchKernelGGL(k_centre_partial, dim3(S), dim3(kWave), lds_partial, st, s.F, n, k, labels, K, rps,
                           s.psum, s.pcnt);
        CD_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_centre_final, dim3((unsigned)ceil_div(K * k, 32)), dim3(256), 0, st, s.psum, s.pcnt,
                           S, K, k, centres);
        CD_LAUNCH_CHECK();
        CD_HIP(hipMemcpyAsync(hchg, s.changed, sizeof(int), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        if (*hchg == 0) break;
    }
    // inertia: squared distances of the rows to the final centres of their labels
    switch (KP) {
        case 8: hipLaunchKernelGGL(k_label_dist<8>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, labels, s.mind); break;
        case 16: hipLaunchKernelGGL(k_label_dist<16>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, labels, s.mind); break;
        case 32: hipLaunchKernelGGL(k_label_dist<32>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, labels, s.mind); break;
        default: hipLaunchKernelGGL(k_label_dist<64>, dim3(B), dim3(kRowsTpb), 0, st, s.F, n, k, centres, labels, s.mind); break;
    }
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_partial, dim3(S), dim3(256), 0, st, s.mind, n, rps, s.dsum);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, s.dsum, S, s.out);
    CD_LAUNCH_CHECK();
    double *hin = reinterpret_cast<double *>(hchg + 2);
    CD_HIP(hipMemcpyAsync(hin, s.out, sizeof(double), hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    if (rounds) *rounds = r;
    if (inertia) *inertia = *hin;
    return CHEBDAV_OK;
}

}  // namespace chebdav
