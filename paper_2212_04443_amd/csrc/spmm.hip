// Fused sparse step of the Chebyshev filter (Alg. 3) and the filter driver.
//
//   Y = alpha * dinv .* (S (dinv .* U)) + beta * U + gamma * Z
//
// S is the binary CSR pattern (Eq. 1), so a row of the product is the
// dinv-weighted sum of the neighbours' rows of U.  Dense blocks are row-major,
// so one neighbour row (w elements) is one contiguous run of w * sizeof(T)
// bytes.  Mapping: a "group" of G lanes owns one matrix row; each lane holds a
// VE-wide vector of columns (16 bytes for the vector path), so a wavefront
// gathers 64/G neighbour rows with one load instruction per lane.  The group
// loads up to G column indices and their dinv values cooperatively (coalesced)
// and broadcasts them lane to lane; neighbour sums run in ascending column
// order, so results are deterministic.  Each of the eight XCDs walks its own
// contiguous range of rows (the gathered rows of block-structured graphs then
// stay in that XCD's L2); the ranges are balanced by nonzeros, so graphs whose
// degrees vary along the node order (power laws, hubs first) keep every XCD busy.
// Inside the filter the work blocks are kept scaled by s = dinv (1 on isolated
// rows), so all steps after the first gather neighbour rows without their dinv
// (one gathered stream per neighbour instead of two).
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

template <typename T, int VE>
struct VecT;
template <>
struct VecT<float, 4> {
    using type = float4;
};
template <>
struct VecT<float, 1> {
    using type = float;
};
template <>
struct VecT<double, 2> {
    using type = double2;
};
template <>
struct VecT<double, 1> {
    using type = double;
};

template <typename T, int VE>
__device__ inline void load_vec(const T *p, T (&v)[VE]) {
    using VT = typename VecT<T, VE>::type;
    const VT x = *reinterpret_cast<const VT *>(p);
    static_assert(sizeof(VT) == VE * sizeof(T), "vector size");
    __builtin_memcpy(v, &x, sizeof(VT));
}

// Neighbour chunk: CH column indices per group per round (each lane of the group
// holds CH/G of them); the chunk's neighbour rows are requested UNR at a time, all
// UNR before any of them is consumed, the next chunk's indices are requested
// before this chunk's rows, and the row's own U and Z entries are requested
// before the neighbour loop.
// DEEP: 16 neighbour rows in flight per batch instead of 8 (fewer waves fit,
// more requests each): faster when the gathered block lives in HBM, slower when
// it fits in the caches.
template <int G, bool DEEP>
struct Chunk {
    static constexpr int CH = G >= 16 ? G : 16;
    static constexpr int PER = CH / G;
    static constexpr int UNR = CH < (DEEP ? 16 : 8) ? CH : (DEEP ? 16 : 8);
};

// NBR = true: the neighbour rows are scaled by their dinv (the plain product),
// streamed per nonzero from nval (CSR order) with the column indices;
// NBR = false: the block is already scaled by s = dinv (1 on isolated rows), so
// the neighbour rows are summed as they are and the row sum takes dinv_i^2.
// flags (kStep*): the output times s_i or divided by s_i, Z times s_i.
template <typename T, typename TO, int VE, int G, bool NBR, bool DEEP>
__global__ void __launch_bounds__(kBlock)
    k_cheb_step(int64_t n, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                const double *__restrict__ nval, const T *__restrict__ dinv, T alpha, T beta, T gamma,
                const T *__restrict__ U,
                int64_t ldu, const T *__restrict__ Z, int64_t ldz, TO *__restrict__ Y, int64_t ldy,
                int w, XcdRanges xr, int flags) {
    constexpr int GPB = kBlock / G;  // rows per block
    constexpr int CH = Chunk<G, DEEP>::CH, PER = Chunk<G, DEEP>::PER, UNR = Chunk<G, DEEP>::UNR;
    const int lane = lane_id();
    const int gl = lane & (G - 1);
    // XCD-aware mapping: consecutive hardware block ids alternate over the eight
    // XCDs, so block b runs on XCD b mod 8; that XCD walks its own contiguous row
    // range (balanced by nonzeros at graph build) in order, block b / 8 next.
    const int xcd = blockIdx.x % kXcds;
    const int64_t r = xr.b[xcd] + (int64_t)(blockIdx.x / kXcds) * GPB + threadIdx.x / G;
    if (r >= xr.b[xcd + 1]) return;  // uniform within a group
    const int c0 = gl * VE;
    const bool active = c0 < w;
    const int64_t beg = row_ptr[r], end = row_ptr[r + 1];

    T ur[VE], zr[VE], acc[VE];
#pragma unroll
    for (int e = 0; e < VE; ++e) {
        ur[e] = T(0);
        zr[e] = T(0);
        acc[e] = T(0);
    }
    if (active && beta != T(0)) load_vec<T, VE>(U + r * ldu + c0, ur);
    if (active && Z != nullptr) load_vec<T, VE>(Z + r * ldz + c0, zr);
    const T di = dinv[r];

    int jl[PER];
    T dl[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t idx = beg + gl + (int64_t)k * G;
        jl[k] = idx < end ? col[idx] : 0;
        if constexpr (NBR) dl[k] = idx < end ? (T)nval[idx] : T(0);
    }
    for (int64_t base = beg; base < end; base += CH) {
        const int cnt = (int)min<int64_t>(CH, end - base);
        int jn[PER];
        T dn[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int64_t nidx = base + CH + gl + (int64_t)k * G;
            jn[k] = nidx < end ? col[nidx] : 0;
            if constexpr (NBR) dn[k] = nidx < end ? (T)nval[nidx] : T(0);
        }
        for (int t0 = 0; t0 < cnt; t0 += UNR) {
            T u[UNR][VE];
#pragma unroll
            for (int i = 0; i < UNR; ++i) {
                const int t = t0 + i;
                const int j = __shfl(jl[(t / G) % PER], t % G, G);
                if (active && t < cnt) {
                    load_vec<T, VE>(U + (int64_t)j * ldu + c0, u[i]);
                } else {
#pragma unroll
                    for (int e = 0; e < VE; ++e) u[i][e] = T(0);
                }
            }
#pragma unroll
            for (int i = 0; i < UNR; ++i) {
                if constexpr (NBR) {
                    const int t = t0 + i;
                    const T dj = __shfl(dl[(t / G) % PER], t % G, G);
#pragma unroll
                    for (int e = 0; e < VE; ++e) acc[e] += dj * u[i][e];
                } else {
#pragma unroll
                    for (int e = 0; e < VE; ++e) acc[e] += u[i][e];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            jl[k] = jn[k];
            if constexpr (NBR) dl[k] = dn[k];
        }
    }
    if (!active) return;
    TO *yp = Y + r * ldy + c0;
    const T si = di > T(0) ? di : T(1);
    const T a_i = NBR ? alpha * di : alpha * (di * di);
    const T g_i = (flags & kStepZMulS) ? gamma * si : gamma;
    T y[VE];
#pragma unroll
    for (int e = 0; e < VE; ++e) {
        T v = a_i * acc[e] + beta * ur[e] + g_i * zr[e];
        if (flags & kStepOutMulS) v *= si;
        if (flags & kStepOutDivS) v /= si;
        y[e] = v;
    }
    if constexpr (sizeof(TO) == sizeof(T)) {
        using VT = typename VecT<T, VE>::type;
        VT v;
        __builtin_memcpy(&v, y, sizeof(VT));
        *reinterpret_cast<VT *>(yp) = v;
    } else {
#pragma unroll
        for (int e = 0; e < VE; ++e) yp[e] = (TO)y[e];
    }
}

template <typename T, typename TO, int VE, bool NBR>
chebdav_status launch_ve(const Graph *g, const T *dinv, T a, T b, T c, const T *U, int64_t ldu,
                         const T *Z, int64_t ldz, TO *Y, int64_t ldy, int w, int flags, hipStream_t st) {
    int lanes = (w + VE - 1) / VE;
    int G = 1;
    while (G < lanes) G <<= 1;
    const int64_t rows_per_block = kBlock / G;
    XcdRanges xr;
    int64_t most = 0;
    for (int x = 0; x <= kXcds; ++x) xr.b[x] = g->xcd_row[x];
    for (int x = 0; x < kXcds; ++x) most = std::max<int64_t>(most, xr.b[x + 1] - xr.b[x]);
    const int64_t grid = std::max<int64_t>(1, ceil_div(most, rows_per_block)) * kXcds;
    if (grid > INT32_MAX) return fail(CHEBDAV_EUNSUPPORTED, "grid too large");
    const dim3 gr((unsigned)grid), bl(kBlock);
    // deeper batches once the gathered block is larger than the 256 MB Infinity
    // Cache (measured: 4 % faster on an 8M-node graph, 11 % slower at 200k nodes)
    const bool deep = G >= 8 && (double)g->n * w * sizeof(T) > 256.0 * 1024 * 1024;
#define CD_CASE(GG, DP)                                                                                 \
    case GG:                                                                                            \
        hipLaunchKernelGGL((k_cheb_step<T, TO, VE, GG, NBR, DP>), gr, bl, 0, st, g->n, g->row_ptr, g->col, \
                           g->nval, dinv, a, b, c, U, ldu, Z, ldz, Y, ldy, w, xr, flags);               \
        break;
    if (deep) {
        switch (G) {
            CD_CASE(8, true)
            CD_CASE(16, true)
            CD_CASE(32, true)
            CD_CASE(64, true)
            default:
                return fail(CHEBDAV_EUNSUPPORTED, "panel too wide");
        }
    } else {
        switch (G) {
            CD_CASE(1, false)
            CD_CASE(2, false)
            CD_CASE(4, false)
            CD_CASE(8, false)
            CD_CASE(16, false)
            CD_CASE(32, false)
            CD_CASE(64, false)
            default:
                return fail(CHEBDAV_EUNSUPPORTED, "panel too wide");
        }
    }
#undef CD_CASE
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

template <typename T, typename TO>
chebdav_status launch_cheb_step(const Graph *g, double alpha, double beta, double gamma,
                                const T *U, int64_t ldu, const T *Z, int64_t ldz, TO *Y,
                                int64_t ldy, int w, hipStream_t st, int flags) {
    if (w < 1) return fail(CHEBDAV_EINVAL, "block width must be >= 1");
    if (ldu < w || ldy < w || (Z && ldz < w)) return fail(CHEBDAV_EINVAL, "leading dimension < width");
    if (!U || !Y) return fail(CHEBDAV_EINVAL, "NULL block");
    if (gamma != 0.0 && !Z) return fail(CHEBDAV_EINVAL, "Z is NULL but gamma != 0");
    const T *dinv;
    if constexpr (sizeof(T) == 8)
        dinv = g->dinv;
    else
        dinv = g->dinv32;
    constexpr int V = 16 / sizeof(T);
    const T a = (T)alpha, b = (T)beta, c = (T)gamma;
    const T *Zp = (gamma != 0.0) ? Z : nullptr;
    for (int c0 = 0; c0 < w; c0 += 64 * V) {
        const int pw = std::min(64 * V, w - c0);
        const bool vec = (pw % V == 0) && (ldu % V == 0) && (ldy % V == 0) &&
                         (!Zp || ldz % V == 0) && aligned(U + c0, 16) && aligned(Y + c0, 16) &&
                         (!Zp || aligned(Zp + c0, 16));
        const T *Zc = Zp ? Zp + c0 : nullptr;
        const bool scaled = (flags & kStepScaled) != 0;
        if (vec) {
            if (scaled)
                CD_TRY((launch_ve<T, TO, V, false>(g, dinv, a, b, c, U + c0, ldu, Zc, ldz, Y + c0, ldy, pw, flags, st)));
            else
                CD_TRY((launch_ve<T, TO, V, true>(g, dinv, a, b, c, U + c0, ldu, Zc, ldz, Y + c0, ldy, pw, flags, st)));
        } else {
            for (int s = 0; s < pw; s += 64) {
                const int sw = std::min(64, pw - s);
                if (scaled)
                    CD_TRY((launch_ve<T, TO, 1, false>(g, dinv, a, b, c, U + c0 + s, ldu, Zp ? Zc + s : nullptr, ldz,
                                                       Y + c0 + s, ldy, sw, flags, st)));
                else
                    CD_TRY((launch_ve<T, TO, 1, true>(g, dinv, a, b, c, U + c0 + s, ldu, Zp ? Zc + s : nullptr, ldz,
                                                      Y + c0 + s, ldy, sw, flags, st)));
            }
        }
    }
    return CHEBDAV_OK;
}

template chebdav_status launch_cheb_step<double, double>(const Graph *, double, double, double,
                                                         const double *, int64_t, const double *,
                                                         int64_t, double *, int64_t, int, hipStream_t, int);
template chebdav_status launch_cheb_step<float, float>(const Graph *, double, double, double,
                                                       const float *, int64_t, const float *,
                                                       int64_t, float *, int64_t, int, hipStream_t, int);
template chebdav_status launch_cheb_step<float, double>(const Graph *, double, double, double,
                                                        const float *, int64_t, const float *,
                                                        int64_t, double *, int64_t, int, hipStream_t, int);

// ---------------------------------------------------------------------------
// Filter driver (Alg. 3).  With c = (cut+upper)/2, e = (upper-cut)/2,
// sigma_1 = e/(scale_pt - c), tau = 2/sigma_1:
//   U_1 = (A X - c X) sigma_1 / e
//   U_k = 2 sigma_k/e (A U_{k-1} - c U_{k-1}) - sigma_{k-1} sigma_k U_{k-2},
//         sigma_k = 1/(tau - sigma_{k-1}),   U_0 = X.
// Since A U = U - dinv .* S (dinv .* U), each step is one fused sparse step with
//   alpha = -s/e, beta = s(1-c)/e, gamma = -sigma_{k-1} sigma_k (s = 2 sigma_k,
//   and s = sigma_1, gamma = 0 for the first step).
// Buffers: three rotating n x kb work blocks; the last step writes Y.
// ---------------------------------------------------------------------------
size_t filter_ws_bytes(int64_t n, int kb, chebdav_dtype dt) {
    const size_t es = dt == CHEBDAV_F32 ? 4 : 8;
    const size_t blk = align_up((size_t)n * kb * es, 256);
    return blk * (dt == CHEBDAV_F32 ? 4 : 3);
}

namespace {
template <typename T>
chebdav_status filter_impl(const Graph *g, const T *x0, int64_t ldx0, double *Y, int64_t ldy,
                           int kb, int m, double cut, double upper, double scale_pt, T *bufs[3],
                           hipStream_t st, bool x_scaled) {
    const double e = (upper - cut) / 2.0;
    const double c = (upper + cut) / 2.0;
    double sigma = e / (scale_pt - c);
    const double tau = 2.0 / sigma;
    const int64_t ldb = kb;
    // The work blocks hold s .* U_k (s = dinv, 1 on isolated rows): A = I - diag(s)
    // S diag(s), so s .* (A U) = s .* U - s^2 .* (S (s .* U)) and the steps after the
    // first gather unscaled rows (no per-neighbour dinv).  The first step scales
    // its output, the second scales its Z = X, the last divides its output by s;
    // with x_scaled (x0 = s .* X) the first two are steps like the others.
    // step 1
    {
        const double al = -sigma / e, be = sigma * (1.0 - c) / e;
        if (m == 1)
            return launch_cheb_step<T, double>(g, al, be, 0.0, x0, ldx0, nullptr, 0, Y, ldy, kb, st,
                                               x_scaled ? (kStepScaled | kStepOutDivS) : 0);
        CD_TRY((launch_cheb_step<T, T>(g, al, be, 0.0, x0, ldx0, nullptr, 0, bufs[0], ldb, kb, st,
                                       x_scaled ? kStepScaled : kStepOutMulS)));
    }
    const T *prev = x0;
    int64_t ldp = ldx0;
    const T *cur = bufs[0];
    for (int k = 2; k <= m; ++k) {
        const double sigma1 = 1.0 / (tau - sigma);
        const double al = -2.0 * sigma1 / e;
        const double be = 2.0 * sigma1 * (1.0 - c) / e;
        const double ga = -sigma * sigma1;
        const int fl = kStepScaled | (k == 2 && !x_scaled ? kStepZMulS : 0);
        if (k == m) {
            CD_TRY((launch_cheb_step<T, double>(g, al, be, ga, cur, ldb, prev, ldp, Y, ldy, kb, st, fl | kStepOutDivS)));
        } else {
            T *out = bufs[(k - 1) % 3];
            CD_TRY((launch_cheb_step<T, T>(g, al, be, ga, cur, ldb, prev, ldp, out, ldb, kb, st, fl)));
            prev = cur;
            ldp = ldb;
            cur = out;
        }
        sigma = sigma1;
    }
    return CHEBDAV_OK;
}
}  // namespace

chebdav_status run_filter(const Graph *g, const double *X, int64_t ldx, double *Y, int64_t ldy,
                          int kb, int m, double cut, double upper, double scale_pt,
                          chebdav_dtype dt, void *ws, size_t ws_bytes, hipStream_t st,
                          hipEvent_t ev_begin, hipEvent_t ev_end, bool x_scaled) {
    if (m < 1 || kb < 1) return fail(CHEBDAV_EINVAL, "need m >= 1 and kb >= 1");
    if (!(scale_pt < cut && cut < upper)) return fail(CHEBDAV_EINVAL, "need scale_pt < cut < upper");
    if (ldx < kb || ldy < kb) return fail(CHEBDAV_EINVAL, "leading dimension < kb");
    if (dt != CHEBDAV_F64 && dt != CHEBDAV_F32) return fail(CHEBDAV_EINVAL, "bad dtype");
    const size_t need = filter_ws_bytes(g->n, kb, dt);
    if (ws_bytes < need || (!ws && need)) return fail(CHEBDAV_ENOMEM, "filter workspace too small (%zu < %zu)", ws_bytes, need);
    const size_t es = dt == CHEBDAV_F32 ? 4 : 8;
    const size_t blk = align_up((size_t)g->n * kb * es, 256);
    char *w = static_cast<char *>(ws);
    if (ev_begin) CD_HIP(hipEventRecord(ev_begin, st));
    if (dt == CHEBDAV_F64) {
        double *b[3] = {reinterpret_cast<double *>(w), reinterpret_cast<double *>(w + blk),
                        reinterpret_cast<double *>(w + 2 * blk)};
        CD_TRY(filter_impl<double>(g, X, ldx, Y, ldy, kb, m, cut, upper, scale_pt, b, st, x_scaled));
    } else {
        float *x32 = reinterpret_cast<float *>(w + 3 * blk);
        CD_TRY((copy_block<double, float>(X, ldx, x32, kb, kb, g->n, st)));
        float *b[3] = {reinterpret_cast<float *>(w), reinterpret_cast<float *>(w + blk),
                       reinterpret_cast<float *>(w + 2 * blk)};
        CD_TRY(filter_impl<float>(g, x32, kb, Y, ldy, kb, m, cut, upper, scale_pt, b, st, x_scaled));
    }
    if (ev_end) CD_HIP(hipEventRecord(ev_end, st));
    return CHEBDAV_OK;
}

}  // namespace chebdav
