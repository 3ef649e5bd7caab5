// Laplacian build (Eq. 1): edge list -> canonical symmetric CSR pattern of S,
// degrees and dinv = 1/sqrt(deg).
//
// Pipeline (all on the device, stream-ordered):
//   count    : validate ids, histogram both endpoints of every non-loop edge
//   scan     : exclusive prefix sum of the counts -> segment offsets
//   scatter  : each endpoint claims a slot in its row segment (integer atomics)
//   sort     : per-row sort + duplicate removal, binned by row length
//              (<= 64: one wavefront, registers + cross-lane bitonic network;
//               <= 4096: one workgroup, bitonic network in LDS;
//               longer: one workgroup, bitonic network in a global scratch row)
//   scan     : prefix sum of the unique counts -> row_ptr
//   compact  : copy unique columns to their final place; deg, dinv, dinv32
// The slot order after `scatter` is nondeterministic, but sorting makes the
// result canonical, so the output is deterministic.
#include <algorithm>
#include <climits>
#include <vector>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kMediumMax = 4096;
constexpr int kLongBlock = 1024;

// RAII device buffer for temporaries of the build.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

__global__ void k_count(const int64_t *__restrict__ edges, int64_t E, int64_t n,
                        int32_t *__restrict__ cnt, int *__restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
        const int64_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            atomicOr(bad, 1);
            continue;
        }
        if (u == v) continue;
        atomicAdd(&cnt[u], 1);
        atomicAdd(&cnt[v], 1);
    }
}

// ---- exclusive scan int32[n] -> int64[n+1] (three phases)
__global__ void k_scan_reduce(const int32_t *__restrict__ in, int64_t n, int64_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        const int64_t k = base + i;
        if (k < n) s += in[k];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s;
}

__global__ void k_scan_bsums(int64_t *__restrict__ bsum, int64_t nb) {
    __shared__ int64_t carry_sh;
    if (threadIdx.x == 0) carry_sh = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < nb ? bsum[k] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, &tot);
        const int64_t carry = carry_sh;
        if (k < nb) bsum[k] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry_sh = carry + tot;
        __syncthreads();
    }
}

__global__ void k_scan_final(const int32_t *__restrict__ in, int64_t n,
                             const int64_t *__restrict__ boff, int64_t *__restrict__ out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t k = base + i;
        v[i] = k < n ? in[k] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = boff[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t k = base + i;
        if (k < n) out[k] = run;
        run += v[i];
        if (k == n - 1) out[n] = run;
    }
}

// ---- scatter both endpoints into their row segments
__global__ void k_scatter(const int64_t *__restrict__ edges, int64_t E,
                          const int64_t *__restrict__ off, int32_t *__restrict__ cur,
                          int32_t *__restrict__ buf) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += stride) {
        const int64_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v) continue;  // ids were validated by k_count
        const int32_t pu = atomicAdd(&cur[u], 1);
        buf[off[u] + pu] = (int32_t)v;
        const int32_t pv = atomicAdd(&cur[v], 1);
        buf[off[v] + pv] = (int32_t)u;
    }
}

// ---- row classification for the sort bins
__global__ void k_classify(const int32_t *__restrict__ cnt, int64_t n, int64_t *__restrict__ med,
                           int64_t *__restrict__ lng, int *__restrict__ counters) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        const int L = cnt[r];
        if (L <= kWave) continue;
        if (L <= kMediumMax)
            med[atomicAdd(&counters[0], 1)] = r;
        else
            lng[atomicAdd(&counters[1], 1)] = r;
    }
}

// Rows of length <= 64: one wavefront per row, one element per lane.
__global__ void k_sort_small(const int64_t *__restrict__ off, const int32_t *__restrict__ cnt,
                             int32_t *__restrict__ buf, int32_t *__restrict__ ucnt, int64_t n) {
    const int lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= n) return;
    const int L = cnt[r];
    if (L > kWave) return;
    const int64_t o = off[r];
    int v = lane < L ? buf[o + lane] : INT_MAX;
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int other = __shfl_xor(v, j, kWave);
            const bool asc = (lane & k) == 0;
            const bool lower = (lane & j) == 0;
            v = (lower == asc) ? min(v, other) : max(v, other);
        }
    }
    const int prev = __shfl_up(v, 1, kWave);
    const bool keep = lane < L && (lane == 0 || v != prev);
    const uint64_t mask = __ballot(keep);
    const int pos = __popcll(mask & ((1ull << lane) - 1ull));
    if (keep) buf[o + pos] = v;
    if (lane == 0) ucnt[r] = __popcll(mask);
}

__device__ inline int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Rows of length in (64, 4096]: one workgroup of 256 per row, sort in LDS.
__global__ void __launch_bounds__(256) k_sort_medium(const int64_t *__restrict__ rows,
                                                     const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ cnt,
                                                     int32_t *__restrict__ buf,
                                                     int32_t *__restrict__ ucnt) {
    __shared__ int s[kMediumMax];
    const int64_t r = rows[blockIdx.x];
    const int L = cnt[r];
    const int64_t o = off[r];
    const int P = next_pow2(L);
    for (int i = threadIdx.x; i < P; i += blockDim.x) s[i] = i < L ? buf[o + i] : INT_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = threadIdx.x; q < P / 2; q += blockDim.x) {
                const int i = 2 * q - (q & (j - 1));
                const int a = s[i], b = s[i + j];
                const bool asc = (i & k) == 0;
                if ((a > b) == asc) {
                    s[i] = b;
                    s[i + j] = a;
                }
            }
            __syncthreads();
        }
    }
    const int chunk = (L + blockDim.x - 1) / blockDim.x;
    const int beg = threadIdx.x * chunk;
    const int end = min(beg + chunk, L);
    int c = 0;
    for (int i = beg; i < end; ++i) c += (i == 0 || s[i] != s[i - 1]);
    int tot;
    int pos = block_excl_scan(c, &tot);
    for (int i = beg; i < end; ++i)
        if (i == 0 || s[i] != s[i - 1]) buf[o + pos++] = s[i];
    if (threadIdx.x == 0) ucnt[r] = tot;
}

// Rows longer than 4096: one workgroup per row, bitonic network in global scratch.
__global__ void __launch_bounds__(kLongBlock) k_sort_long(const int64_t *__restrict__ rows,
                                                          const int64_t *__restrict__ toff,
                                                          const int64_t *__restrict__ off,
                                                          const int32_t *__restrict__ cnt,
                                                          int32_t *__restrict__ buf,
                                                          int32_t *__restrict__ tmp,
                                                          int32_t *__restrict__ ucnt) {
    const int64_t r = rows[blockIdx.x];
    const int64_t L = cnt[r];
    const int64_t o = off[r];
    int32_t *t = tmp + toff[blockIdx.x];
    int64_t P = 1;
    while (P < L) P <<= 1;
    for (int64_t i = threadIdx.x; i < P; i += blockDim.x) t[i] = i < L ? buf[o + i] : INT_MAX;
    __syncthreads();
    for (int64_t k = 2; k <= P; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t q = threadIdx.x; q < P / 2; q += blockDim.x) {
                const int64_t i = 2 * q - (q & (j - 1));
                const int a = t[i], b = t[i + j];
                const bool asc = (i & k) == 0;
                if ((a > b) == asc) {
                    t[i] = b;
                    t[i + j] = a;
                }
            }
            __syncthreads();
        }
    }
    int64_t carry = 0;
    for (int64_t base = 0; base < L; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const int keep = (i < L) && (i == 0 || t[i] != t[i - 1]);
        int tot;
        const int ex = block_excl_scan(keep, &tot);
        if (keep) buf[o + carry + ex] = t[i];
        carry += tot;
    }
    if (threadIdx.x == 0) ucnt[r] = (int32_t)carry;
}

// nval[e] = dinv[col[e]]
__global__ void k_nval(const int32_t *__restrict__ col, const double *__restrict__ dinv, double *__restrict__ nval,
                       int64_t nnz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) nval[e] = dinv[col[e]];
}

// dinv = 1/sqrt(deg) with IEEE round-to-nearest sqrt and division; 0 for deg 0.
__device__ inline double dinv_of(int32_t d) { return d > 0 ? 1.0 / sqrt((double)d) : 0.0; }

__global__ void k_dinv_table(const int32_t *__restrict__ deg, double *__restrict__ dinv, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dinv[i] = dinv_of(deg[i]);
}

// Final placement + degree scaling.  Each wavefront walks rows with a grid
// stride (lanes over a row's columns) and keeps its isolated-row count and
// largest degree in registers: one pair of atomics per wavefront, not per row
// (200k same-address atomics serialize to milliseconds).
__global__ void k_compact(const int64_t *__restrict__ off, const int32_t *__restrict__ ucnt,
                          const int32_t *__restrict__ buf, const int64_t *__restrict__ row_ptr,
                          int32_t *__restrict__ col, int32_t *__restrict__ deg,
                          double *__restrict__ dinv, float *__restrict__ dinv32, int64_t n,
                          int *__restrict__ stats) {
    const int lane = lane_id();
    const int64_t wpb = blockDim.x / kWave;
    const int64_t stride = (int64_t)gridDim.x * wpb;
    int zeros = 0, mx = 0;
    for (int64_t r = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; r < n; r += stride) {
        const int L = ucnt[r];
        const int64_t src = off[r], dst = row_ptr[r];
        for (int i = lane; i < L; i += kWave) col[dst + i] = buf[src + i];
        if (lane == 0) {
            deg[r] = L;
            const double di = dinv_of(L);
            dinv[r] = di;
            dinv32[r] = (float)di;
        }
        zeros += L == 0;
        mx = max(mx, L);
    }
    if (lane == 0) {
        if (zeros) atomicAdd(&stats[0], zeros);
        if (mx) atomicMax(&stats[1], mx);
    }
}

// Row boundaries that split the cost row_ptr[r] + 4 r into eight equal parts
// (binary search over the monotone cost).
__global__ void k_xcd_split(const int64_t *__restrict__ row_ptr, int64_t n, int64_t *__restrict__ out) {
    const int x = threadIdx.x;
    if (x > 8) return;
    const int64_t total = row_ptr[n] + 4 * n;
    const int64_t target = total / 8 * x + (total % 8) * x / 8;
    int64_t lo = 0, hi = n;  // first r with cost(r) >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (row_ptr[mid] + 4 * mid < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    out[x] = x == 8 ? n : lo;
}

chebdav_status scan_counts(const int32_t *in, int64_t n, int64_t *out, int64_t *bsum,
                           hipStream_t st) {
    const int64_t nb = ceil_div(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(1024), 0, st, bsum, nb);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum, out);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

template <class T>
chebdav_status dev_alloc(DevBuf &b, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&b.p, count * sizeof(T));
    if (e != hipSuccess) return fail(CHEBDAV_ENOMEM, "hipMalloc(%zu bytes) failed", count * sizeof(T));
    return CHEBDAV_OK;
}

}  // namespace

chebdav_status dinv_table(const int32_t *deg, double *dinv, int64_t n, hipStream_t st) {
    if (n <= 0) return CHEBDAV_OK;
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536);
    hipLaunchKernelGGL(k_dinv_table, dim3(grid), dim3(256), 0, st, deg, dinv, n);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

void free_graph(Graph *g) {
    if (!g) return;
    if (g->row_ptr) (void)hipFree(g->row_ptr);
    if (g->col) (void)hipFree(g->col);
    if (g->deg) (void)hipFree(g->deg);
    if (g->dinv) (void)hipFree(g->dinv);
    if (g->dinv32) (void)hipFree(g->dinv32);
    if (g->nval) (void)hipFree(g->nval);
    delete g;
}

chebdav_status build_graph(const int64_t *edges, int64_t E, int64_t n, int on_device,
                           hipStream_t st, Graph **out) {
    if (!out) return fail(CHEBDAV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > INT32_MAX) return fail(CHEBDAV_EINVAL, "n_nodes must be in [1, 2^31-1]");
    if (E < 0 || E > (int64_t(1) << 30)) return fail(CHEBDAV_EINVAL, "n_edges must be in [0, 2^30]");
    if (E > 0 && !edges) return fail(CHEBDAV_EINVAL, "edges is NULL");

    DevBuf d_edges, cnt, off, bsum, buf, cur, ucnt, lists, counters, tmp, toff, stats;
    const int64_t nb = ceil_div(n, kScanTile);
    CD_TRY(dev_alloc<int32_t>(cnt, n));
    CD_TRY(dev_alloc<int64_t>(off, n + 1));
    CD_TRY(dev_alloc<int64_t>(bsum, nb));
    CD_TRY(dev_alloc<int32_t>(cur, n));
    CD_TRY(dev_alloc<int32_t>(ucnt, n));
    CD_TRY(dev_alloc<int64_t>(lists, 2 * n));
    CD_TRY(dev_alloc<int>(counters, 4));
    CD_TRY(dev_alloc<int>(stats, 2));
    CD_TRY(dev_alloc<int32_t>(buf, 2 * E));

    const int64_t *ed = edges;
    if (E > 0 && !on_device) {
        CD_TRY(dev_alloc<int64_t>(d_edges, 2 * E));
        CD_HIP(hipMemcpyAsync(d_edges.p, edges, sizeof(int64_t) * 2 * E, hipMemcpyHostToDevice, st));
        ed = static_cast<const int64_t *>(d_edges.p);
    }
    int32_t *c_cnt = static_cast<int32_t *>(cnt.p);
    int64_t *c_off = static_cast<int64_t *>(off.p);
    int *c_counters = static_cast<int *>(counters.p);
    CD_HIP(hipMemsetAsync(c_cnt, 0, sizeof(int32_t) * n, st));
    CD_HIP(hipMemsetAsync(cur.p, 0, sizeof(int32_t) * n, st));
    CD_HIP(hipMemsetAsync(c_counters, 0, sizeof(int) * 4, st));
    CD_HIP(hipMemsetAsync(stats.p, 0, sizeof(int) * 2, st));

    const unsigned egrid = (unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(E, 256), 1), 65536);
    if (E > 0) {
        hipLaunchKernelGGL(k_count, dim3(egrid), dim3(256), 0, st, ed, E, n, c_cnt, c_counters + 2);
        CD_LAUNCH_CHECK();
    }
    int hflags[4] = {0, 0, 0, 0};
    CD_HIP(hipMemcpyAsync(hflags, c_counters, sizeof(hflags), hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    if (hflags[2]) return fail(CHEBDAV_EINVAL, "edge list holds a node id outside [0, n_nodes)");

    CD_TRY(scan_counts(c_cnt, n, c_off, static_cast<int64_t *>(bsum.p), st));
    int32_t *c_buf = static_cast<int32_t *>(buf.p);
    if (E > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(egrid), dim3(256), 0, st, ed, E, c_off,
                           static_cast<int32_t *>(cur.p), c_buf);
        CD_LAUNCH_CHECK();
    }
    int64_t *med = static_cast<int64_t *>(lists.p);
    int64_t *lng = med + n;
    const unsigned ngrid = (unsigned)std::min<int64_t>(ceil_div(n, 256), 65536);
    hipLaunchKernelGGL(k_classify, dim3(ngrid), dim3(256), 0, st, c_cnt, n, med, lng, c_counters);
    CD_LAUNCH_CHECK();
    int32_t *c_ucnt = static_cast<int32_t *>(ucnt.p);
    const int64_t wave_blocks = ceil_div(n, 4);  // 4 wavefronts of 64 per block
    hipLaunchKernelGGL(k_sort_small, dim3((unsigned)wave_blocks), dim3(256), 0, st, c_off, c_cnt,
                       c_buf, c_ucnt, n);
    CD_LAUNCH_CHECK();
    CD_HIP(hipMemcpyAsync(hflags, c_counters, sizeof(hflags), hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    const int n_med = hflags[0], n_long = hflags[1];
    if (n_med > 0) {
        hipLaunchKernelGGL(k_sort_medium, dim3(n_med), dim3(256), 0, st, med, c_off, c_cnt, c_buf,
                           c_ucnt);
        CD_LAUNCH_CHECK();
    }
    if (n_long > 0) {
        // scratch rows padded to powers of two
        std::vector<int64_t> rows(n_long), lens(n_long), toffs(n_long);
        CD_HIP(hipMemcpyAsync(rows.data(), lng, sizeof(int64_t) * n_long, hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        std::vector<int32_t> cnt_h(1);
        int64_t total = 0;
        for (int i = 0; i < n_long; ++i) {
            CD_HIP(hipMemcpy(cnt_h.data(), c_cnt + rows[i], sizeof(int32_t), hipMemcpyDeviceToHost));
            int64_t P = 1;
            while (P < cnt_h[0]) P <<= 1;
            toffs[i] = total;
            total += P;
        }
        CD_TRY(dev_alloc<int32_t>(tmp, total));
        CD_TRY(dev_alloc<int64_t>(toff, n_long));
        CD_HIP(hipMemcpyAsync(toff.p, toffs.data(), sizeof(int64_t) * n_long, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_sort_long, dim3(n_long), dim3(kLongBlock), 0, st, lng,
                           static_cast<int64_t *>(toff.p), c_off, c_cnt, c_buf,
                           static_cast<int32_t *>(tmp.p), c_ucnt);
        CD_LAUNCH_CHECK();
    }

    Graph *g = new Graph;
    g->n = n;
    auto cleanup = [&]() { free_graph(g); };
    if (hipMalloc(&g->row_ptr, sizeof(int64_t) * (n + 1)) != hipSuccess ||
        hipMalloc(&g->deg, sizeof(int32_t) * n) != hipSuccess ||
        hipMalloc(&g->dinv, sizeof(double) * n) != hipSuccess ||
        hipMalloc(&g->dinv32, sizeof(float) * n) != hipSuccess) {
        cleanup();
        return fail(CHEBDAV_ENOMEM, "graph allocation failed");
    }
    chebdav_status s = scan_counts(c_ucnt, n, g->row_ptr, static_cast<int64_t *>(bsum.p), st);
    if (s != CHEBDAV_OK) {
        cleanup();
        return s;
    }
    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, g->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        cleanup();
        return fail(CHEBDAV_EHIP, "reading nnz failed");
    }
    g->nnz = nnz;
    if (hipMalloc(&g->col, sizeof(int32_t) * std::max<int64_t>(nnz, 1)) != hipSuccess) {
        cleanup();
        return fail(CHEBDAV_ENOMEM, "col allocation failed (%lld entries)", (long long)nnz);
    }
    hipLaunchKernelGGL(k_compact, dim3((unsigned)std::min<int64_t>(wave_blocks, 2048)), dim3(256), 0, st, c_off,
                       c_ucnt, c_buf,
                       g->row_ptr, g->col, g->deg, g->dinv, g->dinv32, n,
                       static_cast<int *>(stats.p));
    int hstats[2] = {0, 0};
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hstats, stats.p, sizeof(hstats), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        cleanup();
        return fail(CHEBDAV_EHIP, "CSR compaction failed");
    }
    g->n_isolated = hstats[0];
    g->max_deg = hstats[1];
    // dinv of every nonzero's column, in CSR order: the plain product streams it
    // with the column indices instead of gathering dinv per neighbour
    if (hipMalloc(&g->nval, sizeof(double) * std::max<int64_t>(nnz, 1)) != hipSuccess) {
        cleanup();
        return fail(CHEBDAV_ENOMEM, "allocation failed (%lld nonzero scalings)", (long long)nnz);
    }
    if (nnz > 0) {
        hipLaunchKernelGGL(k_nval, dim3((unsigned)std::min<int64_t>(ceil_div(nnz, 256), 65536)), dim3(256), 0, st,
                           g->col, g->dinv, g->nval, nnz);
        if (hipGetLastError() != hipSuccess) {
            cleanup();
            return fail(CHEBDAV_EHIP, "nonzero scalings failed");
        }
    }
    // per-XCD row ranges for the sparse step (bsum has room: nb >= 1 entries, use counters' buffer)
    {
        int64_t *d_split = static_cast<int64_t *>(lists.p);  // 2n >= 9 entries unless n < 5
        DevBuf small;
        if (2 * n < 9) {
            if (dev_alloc<int64_t>(small, 9) != CHEBDAV_OK) {
                cleanup();
                return fail(CHEBDAV_ENOMEM, "allocation failed");
            }
            d_split = static_cast<int64_t *>(small.p);
        }
        hipLaunchKernelGGL(k_xcd_split, dim3(1), dim3(64), 0, st, g->row_ptr, n, d_split);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(g->xcd_row, d_split, sizeof(g->xcd_row), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            cleanup();
            return fail(CHEBDAV_EHIP, "XCD split failed");
        }
    }
    *out = g;
    return CHEBDAV_OK;
}

}  // namespace chebdav
