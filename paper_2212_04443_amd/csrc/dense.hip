// Dense FP64 kernels on tall row-major blocks (n rows, few columns):
//   gram     C = Xs^T Y      (Rayleigh-quotient columns, Gram matrices)
//   update   Y = a Xs B + b Y (projections, Cholesky-QR, subspace rotation)
//   colnorms ||X(:,j) - Y(:,j) theta_j||_2 (residuals, column norms)
//   gather_cols / copy_block / fill / philox_fill / check_finite
// Xs is a "two-segment" column range: the locked and active parts of the basis
// are separate arrays, so V(:, 1:ksub) = [Vlocked, Vactive] is read in place.
// Reductions over n are split over row ranges, written to a partial buffer and
// summed in a fixed order, so every result is deterministic.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int TB = 64;   // tile edge (rows / columns of the output tile)
constexpr int NT = 256;  // threads per block of the column-norm kernel

__device__ inline double seg_load(const Seg2 &s, int64_t row, int c) {
    return c < s.p1 ? s.X1[row * s.ld1 + c] : s.X2[row * s.ld2 + (c - s.p1)];
}

typedef double d4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 lane layout (one wavefront; checked on gfx950): A
// (16 x 4) element (i, k) in lane i + 16 k; B (4 x 16) element (k, j) in lane
// j + 16 k; the 16 x 16 result element (i, j) in lane j + 16 (i % 4), register i / 4.
__device__ inline d4_t mfma16x16x4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partial Gram on matrix cores: one wavefront computes the (16 TP) x (16 TQT)
// tile (i0.., j0..) of Xs^T Y over the rows of split z, four rows per MFMA step
// and 4 UR rows per loop trip, with both operands loaded straight from the
// row-major blocks (lane k*16 + c reads column c of row k: four 128-byte row
// segments per load).  The loads of the next trip are issued before the MFMAs
// of the current one (two register sets), so a wavefront always has a trip of
// loads in flight.  TP = 2 serves p <= 32 without idle matrix-core work.
// NWG wavefronts may share a split (trips interleaved between them; their tiles
// are added in wavefront order through LDS before the one store): more loads
// in flight when short blocks leave fewer splits than wavefronts the GPU holds.
template <int TP, int TQT, int UR, int NWG = 1>
__global__ void __launch_bounds__(64 * NWG) k_gram(Seg2 xs, const double *__restrict__ Y, int64_t ldy, int q,
                                                   int64_t n, int64_t rows_per_split, double *__restrict__ part) {
    const int p = xs.cols();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kr = lane >> 4, cc = lane & 15;
    const int i0 = blockIdx.x * (16 * TP), j0 = blockIdx.y * (16 * TQT);
    const int64_t r_beg = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r_end = min(n, r_beg + rows_per_split);
    d4_t acc[TP][TQT];
#pragma unroll
    for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int u = 0; u < TQT; ++u) acc[t][u] = d4_t{0.0, 0.0, 0.0, 0.0};
    bool colv[TP], colw[TQT];
#pragma unroll
    for (int t = 0; t < TP; ++t) colv[t] = i0 + 16 * t + cc < p;
#pragma unroll
    for (int u = 0; u < TQT; ++u) colw[u] = j0 + 16 * u + cc < q;
    auto load = [&](int64_t r, double (&a)[UR][TP], double (&b)[UR][TQT]) {
#pragma unroll
        for (int h = 0; h < UR; ++h) {
            const int64_t row = r + 4 * h + kr;
            const bool rv = row < r_end;
#pragma unroll
            for (int t = 0; t < TP; ++t) a[h][t] = (rv && colv[t]) ? seg_load(xs, row, i0 + 16 * t + cc) : 0.0;
#pragma unroll
            for (int u = 0; u < TQT; ++u) b[h][u] = (rv && colw[u]) ? Y[row * ldy + j0 + 16 * u + cc] : 0.0;
        }
    };
    auto trip = [&](double (&a)[UR][TP], double (&b)[UR][TQT]) {
#pragma unroll
        for (int h = 0; h < UR; ++h)
#pragma unroll
            for (int t = 0; t < TP; ++t)
#pragma unroll
                for (int u = 0; u < TQT; ++u) acc[t][u] = mfma16x16x4(a[h][t], b[h][u], acc[t][u]);
    };
    constexpr int64_t step = 4 * UR, stride = step * NWG;
    double a0[UR][TP], b0[UR][TQT], a1[UR][TP], b1[UR][TQT];
    int64_t r = r_beg + wave * step;
    if (r < r_end) load(r, a0, b0);
    while (r < r_end) {
        const int64_t r1 = r + stride;
        if (r1 < r_end) load(r1, a1, b1);
        trip(a0, b0);
        if (r1 >= r_end) break;
        const int64_t r2 = r1 + stride;
        if (r2 < r_end) load(r2, a0, b0);
        trip(a1, b1);
        r = r2;
    }
    if constexpr (NWG > 1) {
        __shared__ d4_t red[TP * TQT][64];
        for (int w = 1; w < NWG; ++w) {
            if (wave == w) {
#pragma unroll
                for (int t = 0; t < TP; ++t)
#pragma unroll
                    for (int u = 0; u < TQT; ++u) red[t * TQT + u][lane] = acc[t][u];
            }
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int t = 0; t < TP; ++t)
#pragma unroll
                    for (int u = 0; u < TQT; ++u) acc[t][u] += red[t * TQT + u][lane];
            }
            __syncthreads();
        }
        if (wave != 0) return;
    }
    double *out = part + (int64_t)blockIdx.z * p * q;
#pragma unroll
    for (int t = 0; t < TP; ++t)
#pragma unroll
        for (int u = 0; u < TQT; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + 16 * t + kr + 4 * v, j = j0 + 16 * u + cc;
                if (i < p && j < q) out[(int64_t)i * q + j] = acc[t][u][v];
            }
}

// Fixed-order reduction of S partial arrays of E elements.  A block owns EB
// consecutive elements; thread group zg (ZG groups) adds splits z = zg, zg + ZG,
// ... into four accumulators (z mod 4 ZG), combined as (a0 + a1) + (a2 + a3);
// the ZG group sums are then added in order.  The order depends only on S.
// MODE 0 writes C[(e / q) * ldc + e % q] (a Gram tile); MODE 1 writes sqrt(sum) to C[e];
// MODE 2 (square Gram G = X^T X) writes the Newton-Schulz matrix (3 I - G) / 2 in
// the layout of MODE 0 (one step X <- X (3 I - X^T X) / 2 towards the
// orthonormal polar factor when X^T X is close to I).
template <int MODE>
__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ part, int S, int64_t E, int q,
                                                double *__restrict__ C, int64_t ldc) {
    constexpr int EB = 8, ZG = 32;
    __shared__ double sh[ZG][EB];
    const int el = threadIdx.x % EB, zg = threadIdx.x / EB;
    const int64_t e = (int64_t)blockIdx.x * EB + el;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < E) {
        int z = zg;
        for (; z + 3 * ZG < S; z += 4 * ZG) {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += part[(int64_t)(z + u * ZG) * E + e];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u)
            if (z + u * ZG < S) a[u] += part[(int64_t)(z + u * ZG) * E + e];
    }
    sh[zg][el] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (zg == 0 && e < E) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < ZG; ++g) t += sh[g][el];
        if (MODE == 0)
            C[(e / q) * ldc + (e % q)] = t;
        else if (MODE == 1)
            C[e] = sqrt(t);
        else
            C[(e / q) * ldc + (e % q)] = ((e / q) == (e % q) ? 1.5 : 0.0) - 0.5 * t;
    }
}

// Row splits of a Gram product: about 2048 wavefronts in total, at least 256 rows each.
int gram_splits(int64_t n, int p, int q) {
    const int tiles = (int)(ceil_div(p, TB) * ceil_div(q, TB));
    int64_t s = std::max<int64_t>(1, 2048 / tiles);
    s = std::min<int64_t>(s, std::max<int64_t>(1, ceil_div(n, 256)));
    return (int)s;
}

// Y = alpha Xs B + beta Y on matrix cores.  A block of NW wavefronts covers
// 16 TR NW consecutive rows and (16 TQT) columns of Y; each wavefront owns 16 TR
// rows, accumulates over all p columns of Xs and writes its tile only at the
// end, so Y may alias Xs when it has a single column tile.  The reduction index
// runs over 16-column groups of the two segments of Xs (a segment's last group
// is zero-padded), and inside a group it is permuted per lane: lane group kr
// takes columns 2kr, 2kr + 1 and 8 + 2kr, 9 + 2kr, so one 16-byte load per
// lane covers a contiguous 64-byte half of every row's 128-byte group (two
// 8-byte loads when the segment's base or leading dimension is not 16-byte
// aligned).  The rows of B for KC such indices at a time (128 up to 32 columns,
// 64 for 64 columns: 32 KB either way) are staged in LDS,
// shared by the block's wavefronts, and the X loads of the next group are issued
// before the MFMAs of the current one.  Fewer registers per wavefront (B is not
// held in registers) keep 4-8 wavefronts per SIMD resident.
typedef double d2_t __attribute__((ext_vector_type(2)));

template <int TR, int TQT, int NW, int KC>
__global__ void __launch_bounds__(64 * NW) k_update(Seg2 xs, int vec1, int vec2, const double *__restrict__ B,
                                                    int64_t ldb, double alpha, double beta, double *Y, int64_t ldy,
                                                    int q, int64_t n) {
    constexpr int QW = 16 * TQT;
    __shared__ double sB[KC * QW];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kr = lane >> 4, cc = lane & 15;
    const int64_t r0 = ((int64_t)blockIdx.x * NW + wave) * 16 * TR;
    const int j0 = blockIdx.y * QW;
    const int g1 = (xs.p1 + 15) >> 4;                // 16-column groups of segment 1
    const int pv = 16 * (g1 + ((xs.p2 + 15) >> 4));  // padded reduction length
    d4_t acc[TR][TQT];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int u = 0; u < TQT; ++u) acc[t][u] = d4_t{0.0, 0.0, 0.0, 0.0};
    bool rowv[TR];
#pragma unroll
    for (int t = 0; t < TR; ++t) rowv[t] = r0 + 16 * t + cc < n;
    // X(row, v .. v+15) for this lane's two column pairs of group v / 16
    auto xload = [&](int v, d2_t (&a)[TR][2]) {
        const bool s1 = v < 16 * g1;
        const double *base = s1 ? xs.X1 : xs.X2;
        const int64_t ld = s1 ? xs.ld1 : xs.ld2;
        const int pc = s1 ? xs.p1 : xs.p2;
        const int cb = s1 ? v : v - 16 * g1;
        const bool vec = s1 ? vec1 : vec2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = cb + 8 * h + 2 * kr;
#pragma unroll
            for (int t = 0; t < TR; ++t) {
                const double *src = base + (r0 + 16 * t + cc) * ld + c;
                d2_t x = d2_t{0.0, 0.0};
                if (rowv[t] && c + 1 < pc) {
                    if (vec)
                        x = *reinterpret_cast<const d2_t *>(src);
                    else
                        x = d2_t{src[0], src[1]};
                } else if (rowv[t] && c < pc) {
                    x.x = src[0];
                }
                a[t][h] = x;
            }
        }
    };
    // MFMA step s of a group uses reduction index 8 (s >> 1) + 2 kr + (s & 1)
    auto trip = [&](int v, d2_t (&a)[TR][2]) {
        double b[4][TQT];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int e = (v % KC) + 8 * (s >> 1) + 2 * kr + (s & 1);
#pragma unroll
            for (int u = 0; u < TQT; ++u) b[s][u] = sB[e * QW + 16 * u + cc];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < TR; ++t)
#pragma unroll
                for (int u = 0; u < TQT; ++u) acc[t][u] = mfma16x16x4(a[t][s >> 1][s & 1], b[s][u], acc[t][u]);
    };
    d2_t a0[TR][2], a1[TR][2];
    if (pv > 0) xload(0, a0);
    for (int v0 = 0; v0 < pv; v0 += KC) {
        __syncthreads();  // every wavefront is done with the previous chunk
        for (int e = threadIdx.x; e < KC * QW; e += 64 * NW) {
            const int v = v0 + e / QW, j = j0 + e % QW;
            const bool s1 = v < 16 * g1;
            const int c = s1 ? v : v - 16 * g1;
            const bool ok = j < q && (s1 ? c < xs.p1 : (v < pv && c < xs.p2));
            sB[e] = ok ? B[(int64_t)(s1 ? c : xs.p1 + c) * ldb + j] : 0.0;
        }
        __syncthreads();
        // a chunk holds KC / 16 groups, an even number (fewer only in the last
        // chunk), so every chunk but the last starts with its first group in a0
        const int vend = min(pv, v0 + KC);
        for (int v = v0; v < vend; v += 32) {
            if (v + 16 < pv) xload(v + 16, a1);
            trip(v, a0);
            if (v + 16 >= vend) break;
            if (v + 32 < pv) xload(v + 32, a0);
            trip(v + 16, a1);
        }
    }
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = r0 + 16 * t + kr + 4 * r;
            if (row >= n) continue;
#pragma unroll
            for (int u = 0; u < TQT; ++u) {
                const int j = j0 + 16 * u + cc;
                if (j >= q) continue;
                double *y = Y + row * ldy + j;
                *y = beta == 0.0 ? alpha * acc[t][u][r] : alpha * acc[t][u][r] + beta * (*y);
            }
        }
}

// Column sums of squares of (X - Y diag(theta)) over a row range per block.
__global__ void __launch_bounds__(NT) k_colnorm(const double *__restrict__ X, int64_t ldx,
                                                const double *__restrict__ Y, int64_t ldy,
                                                const double *__restrict__ theta, int w, int64_t n,
                                                int64_t rows_per_block, double *__restrict__ part) {
    __shared__ double red[NT];
    const int R = NT / w;  // row lanes (w <= NT)
    const int c = threadIdx.x % w, rr = threadIdx.x / w;
    const int64_t r_beg = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r_end = min(n, r_beg + rows_per_block);
    double s = 0.0;
    if (rr < R) {
        const double th = (Y && theta) ? theta[c] : 0.0;
        for (int64_t r = r_beg + rr; r < r_end; r += R) {
            double v = X[r * ldx + c];
            if (Y) v -= Y[r * ldy + c] * th;
            s += v * v;
        }
    }
    red[threadIdx.x] = (rr < R) ? s : 0.0;
    __syncthreads();
    if (threadIdx.x < w) {
        double t = 0.0;
        for (int k = 0; k < R; ++k) t += red[k * w + threadIdx.x];
        part[(int64_t)blockIdx.x * w + threadIdx.x] = t;
    }
}

constexpr int kColnormBlocks = 1024;

// One wavefront per row: stage the row's selected entries, then write them.
__device__ inline double row_scale(const double *rs, int64_t r) {
    if (!rs) return 1.0;
    const double d = rs[r];
    return d > 0.0 ? d : 1.0;
}

// Up to 64 columns: a wavefront holds 64 / wp rows (wp = w rounded up to a power
// of two), thread (row slot, column c) loads map[c] once and walks the rows with a
// grid stride.  A row never spans two wavefronts, and every lane of a wavefront
// issues its load before any lane stores, so Src may alias Dst.
__global__ void k_gather_cols_packed(const double *Src, int64_t lds, double *Dst, int64_t ldd,
                                     const int32_t *__restrict__ map, int w, int wp_log2, int64_t n,
                                     const double *__restrict__ rs) {
    const int c = threadIdx.x & ((1 << wp_log2) - 1);
    const int slot = threadIdx.x >> wp_log2;
    const int rows_per_block = blockDim.x >> wp_log2;
    const bool active = c < w;
    const int src_c = active ? map[c] : 0;
    for (int64_t r = (int64_t)blockIdx.x * rows_per_block + slot; r < n; r += (int64_t)gridDim.x * rows_per_block) {
        const double v = active ? row_scale(rs, r) * Src[r * lds + src_c] : 0.0;
        if (active) Dst[r * ldd + c] = v;
    }
}

template <int PER_LANE>
__global__ void k_gather_cols(const double *Src, int64_t lds, double *Dst, int64_t ldd,
                              const int32_t *__restrict__ map, int w, int64_t n, const double *__restrict__ rs) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= n) return;
    const int lane = lane_id();
    const double sr = row_scale(rs, r);
    double v[PER_LANE];
#pragma unroll
    for (int t = 0; t < PER_LANE; ++t) {
        const int j = lane + t * kWave;
        v[t] = j < w ? sr * Src[r * lds + map[j]] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < PER_LANE; ++t) {
        const int j = lane + t * kWave;
        if (j < w) Dst[r * ldd + j] = v[t];
    }
}

template <typename TS, typename TD>
__global__ void k_copy_block(const TS *__restrict__ S, int64_t lds, TD *__restrict__ D, int64_t ldd,
                             int w, int64_t n, const double *__restrict__ rs) {
    const int64_t total = n * (int64_t)w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t r = e / w;
        const int c = (int)(e - r * w);
        D[r * ldd + c] = rs ? (TD)(row_scale(rs, r) * (double)S[r * lds + c]) : (TD)S[r * lds + c];
    }
}

__global__ void k_fill(double *__restrict__ p, int64_t count, double v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) p[e] = v;
}

__global__ void k_philox(double *__restrict__ X, int64_t n, int w, int64_t ld, uint64_t seed,
                         uint64_t first_col, const double *__restrict__ rs) {
    const int64_t total = n * (int64_t)w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t r = e / w;
        const int j = (int)(e - r * w);
        const uint64_t q = first_col + (uint64_t)j;
        uint32_t c[4] = {(uint32_t)r, (uint32_t)((uint64_t)r >> 32), (uint32_t)q, 0u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t u = (((uint64_t)c[1] << 32) | c[0]) >> 11;
        const double x = (double)u * 0x1.0p-52 - 1.0;
        X[r * ld + j] = rs ? row_scale(rs, r) * x : x;
    }
}

__global__ void k_check_finite(const double *__restrict__ X, int64_t ld, int w, int64_t n,
                               int *__restrict__ flag) {
    const int64_t total = n * (int64_t)w;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t r = e / w;
        const int c = (int)(e - r * w);
        bad |= !isfinite(X[r * ld + c]);
    }
    if (__any(bad) && lane_id() == 0) atomicOr(flag, 1);
}

unsigned grid_for(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 8192));
}

}  // namespace

// Upper bound of splits * p' * q' over all p' <= p, q' <= q: splits * tiles' <=
// max(tiles', 2048) <= max(tiles, 2048) and p' q' <= tiles' * TB * TB.
size_t gram_partial_elems(int64_t, int p, int q) {
    const int64_t tiles = ceil_div(std::max(p, 1), TB) * ceil_div(std::max(q, 1), TB);
    return (size_t)std::max<int64_t>(tiles, 2048) * TB * TB;
}

chebdav_status gram(const Seg2 &Xs, const double *Y, int64_t ldy, int q, int64_t n, double *C,
                    int64_t ldc, double *partial, hipStream_t st, bool ns) {
    const int p = Xs.cols();
    if (p == 0 || q == 0) return CHEBDAV_OK;
    const int splits = gram_splits(n, p, q);
    const int64_t rps = ceil_div(ceil_div(n, splits), 16) * 16;
    const int qt = std::min(q, TB);
    const int pt = p <= 32 ? 32 : TB;  // X tile: 32 or 64 columns
    const dim3 grid((unsigned)ceil_div(p, pt), (unsigned)ceil_div(q, qt), (unsigned)splits);
    // one tile and fewer row splits than the 2048 wanted (short blocks): two
    // wavefronts per split where measured faster (tiles of at most 64 x 32 or
    // 32 x 64: 20-25 % at 200k rows; 64 x 64 tiles lose)
    const bool pair = grid.x * grid.y == 1 && splits < 2048;
    if (pt == 32) {
        if (qt <= 16)
            hipLaunchKernelGGL((k_gram<2, 1, 4>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else if (qt <= 32 && pair)
            hipLaunchKernelGGL((k_gram<2, 2, 4, 2>), grid, dim3(128), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else if (qt <= 32)
            hipLaunchKernelGGL((k_gram<2, 2, 4>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else if (pair)
            hipLaunchKernelGGL((k_gram<2, 4, 2, 2>), grid, dim3(128), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else
            hipLaunchKernelGGL((k_gram<2, 4, 2>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
    } else {
        if (qt <= 16)
            hipLaunchKernelGGL((k_gram<4, 1, 4>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else if (qt <= 32 && pair)
            hipLaunchKernelGGL((k_gram<4, 2, 2, 2>), grid, dim3(128), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else if (qt <= 32)
            hipLaunchKernelGGL((k_gram<4, 2, 2>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
        else
            hipLaunchKernelGGL((k_gram<4, 4, 2>), grid, dim3(64), 0, st, Xs, Y, ldy, q, n, rps, partial);
    }
    CD_LAUNCH_CHECK();
    const int64_t pq = (int64_t)p * q;
    if (ns && p != q) return fail(CHEBDAV_EINVAL, "Newton-Schulz matrix of a non-square Gram product");
    if (ns)
        hipLaunchKernelGGL(k_reduce<2>, dim3((unsigned)ceil_div(pq, 8)), dim3(256), 0, st, partial, splits, pq,
                           q, C, ldc);
    else
        hipLaunchKernelGGL(k_reduce<0>, dim3((unsigned)ceil_div(pq, 8)), dim3(256), 0, st, partial, splits, pq,
                           q, C, ldc);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

int update_max_inplace_cols() { return TB; }

chebdav_status update(const Seg2 &Xs, const double *B, int64_t ldb, double alpha, double beta,
                      double *Y, int64_t ldy, int q, int64_t n, hipStream_t st) {
    if (q == 0 || n == 0) return CHEBDAV_OK;
    if (Xs.cols() == 0) {
        if (beta == 1.0) return CHEBDAV_OK;
        return fail(CHEBDAV_EUNSUPPORTED, "update with an empty basis");
    }
    auto vec_ok = [](const double *X, int64_t ld) {
        return (reinterpret_cast<uintptr_t>(X) % 16) == 0 && ld % 2 == 0;
    };
    const int vec1 = Xs.p1 > 0 && vec_ok(Xs.X1, Xs.ld1);
    const int vec2 = Xs.p2 > 0 && vec_ok(Xs.X2, Xs.ld2);
    const int qt = std::min(q, TB);
    const unsigned gy = (unsigned)ceil_div(q, qt);
    // rows per block: 16 TR NW (measured best: TR = 1 up to 32 columns, TR = 2 for 64; NW = 8;
    // KC = 128 is 2-5 % faster than 64 up to 32 columns, equal at 64)
    if (qt <= 16) {
        const dim3 grid((unsigned)ceil_div(n, 256), gy);
        hipLaunchKernelGGL((k_update<2, 1, 8, 128>), grid, dim3(512), 0, st, Xs, vec1, vec2, B, ldb, alpha, beta, Y, ldy, q, n);
    } else if (qt <= 32) {
        const dim3 grid((unsigned)ceil_div(n, 128), gy);
        hipLaunchKernelGGL((k_update<1, 2, 8, 128>), grid, dim3(512), 0, st, Xs, vec1, vec2, B, ldb, alpha, beta, Y, ldy, q, n);
    } else {
        const dim3 grid((unsigned)ceil_div(n, 256), gy);
        hipLaunchKernelGGL((k_update<2, 4, 8, 64>), grid, dim3(512), 0, st, Xs, vec1, vec2, B, ldb, alpha, beta, Y, ldy, q, n);
    }
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

size_t colnorm_partial_elems(int64_t, int w) { return (size_t)kColnormBlocks * std::max(w, 1); }

chebdav_status colnorms(const double *X, int64_t ldx, const double *Y, int64_t ldy,
                        const double *theta, int w, int64_t n, double *out, double *partial,
                        hipStream_t st) {
    if (w == 0) return CHEBDAV_OK;
    for (int c0 = 0; c0 < w; c0 += NT) {
        const int pw = std::min(NT, w - c0);
        const int blocks = (int)std::min<int64_t>(kColnormBlocks, std::max<int64_t>(1, ceil_div(n, 256)));
        const int64_t rpb = ceil_div(n, blocks);
        hipLaunchKernelGGL(k_colnorm, dim3(blocks), dim3(NT), 0, st, X + c0, ldx, Y ? Y + c0 : nullptr,
                           ldy, theta ? theta + c0 : nullptr, pw, n, rpb, partial);
        CD_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_reduce<1>, dim3((unsigned)ceil_div(pw, 8)), dim3(256), 0, st, partial, blocks,
                           (int64_t)pw, 1, out + c0, 1);
        CD_LAUNCH_CHECK();
    }
    return CHEBDAV_OK;
}

chebdav_status gather_cols(const double *Src, int64_t lds, double *Dst, int64_t ldd,
                           const int32_t *map, int w, int64_t n, hipStream_t st, const double *rs) {
    if (w == 0 || n == 0) return CHEBDAV_OK;
    const unsigned grid = (unsigned)ceil_div(n, 4);
    if (w <= 64) {
        int lg = 0;
        while ((1 << lg) < w) ++lg;
        const int64_t rows_per_block = 256 >> lg;
        const unsigned pg = (unsigned)std::min<int64_t>(ceil_div(n, rows_per_block), 4096);
        hipLaunchKernelGGL(k_gather_cols_packed, dim3(pg), dim3(256), 0, st, Src, lds, Dst, ldd, map, w, lg, n, rs);
    } else if (w <= 128)
        hipLaunchKernelGGL(k_gather_cols<2>, dim3(grid), dim3(256), 0, st, Src, lds, Dst, ldd, map, w, n, rs);
    else if (w <= 256)
        hipLaunchKernelGGL(k_gather_cols<4>, dim3(grid), dim3(256), 0, st, Src, lds, Dst, ldd, map, w, n, rs);
    else if (w <= 512)
        hipLaunchKernelGGL(k_gather_cols<8>, dim3(grid), dim3(256), 0, st, Src, lds, Dst, ldd, map, w, n, rs);
    else
        return fail(CHEBDAV_EUNSUPPORTED, "gather of more than 512 columns");
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

template <typename TS, typename TD>
chebdav_status copy_block(const TS *Src, int64_t lds, TD *Dst, int64_t ldd, int w, int64_t n,
                          hipStream_t st, const double *rs) {
    if (w == 0 || n == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL((k_copy_block<TS, TD>), dim3(grid_for(n * w)), dim3(256), 0, st, Src, lds, Dst,
                       ldd, w, n, rs);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}
template chebdav_status copy_block<double, double>(const double *, int64_t, double *, int64_t, int,
                                                   int64_t, hipStream_t, const double *);
template chebdav_status copy_block<double, float>(const double *, int64_t, float *, int64_t, int,
                                                  int64_t, hipStream_t, const double *);
template chebdav_status copy_block<float, double>(const float *, int64_t, double *, int64_t, int,
                                                  int64_t, hipStream_t, const double *);

chebdav_status fill_f64(double *p, int64_t count, double v, hipStream_t st) {
    if (count == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(256), 0, st, p, count, v);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

chebdav_status philox_fill(double *X, int64_t n, int w, int64_t ld, uint64_t seed,
                           uint64_t first_col, hipStream_t st, const double *rs) {
    if (w == 0 || n == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL(k_philox, dim3(grid_for(n * w)), dim3(256), 0, st, X, n, w, ld, seed, first_col, rs);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

chebdav_status check_finite(const double *X, int64_t ld, int w, int64_t n, int *flag,
                            hipStream_t st) {
    if (w == 0 || n == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n * w)), dim3(256), 0, st, X, ld, w, n, flag);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
