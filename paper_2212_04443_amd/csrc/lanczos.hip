// Lanczos estimate of the spectrum bounds of A (Sec. 2: when the filter's
// bounds are unknown, a few Lanczos steps estimate them).
//
// Plain Lanczos (no reorthogonalization) from Philox column 2^32 - 1 of the
// seed, scaled to unit length:
//   w = A v_j - beta_{j-1} v_{j-1}   (one fused sparse step)
//   alpha_j = v_j . w;  w -= alpha_j v_j;  beta_j = ||w||;  v_{j+1} = w / beta_j
// stopping early when beta_j <= 1e-12 max(1, |alpha_j|).  The Ritz values of
// the tridiagonal T_k come from the small eigensolver; the bounds (Zhou & Li,
// 2011) are max Ritz + beta_k and min Ritz - beta_k.  The host reads alpha_j and
// beta_j after every step (the next sparse step takes beta_j as a scalar).
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_util.h"
#include "internal.h"

namespace chebdav {

void *pinned_host(size_t bytes, int slot);

namespace {

constexpr uint64_t kStartColumn = 0xFFFFFFFFull;
constexpr int kMaxSteps = 256;

// w -= a[0] v
__global__ void k_axpy_dev(double *__restrict__ w, const double *__restrict__ v, const double *__restrict__ a,
                           int64_t n) {
    const double s = a[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) w[i] -= s * v[i];
}

// y = x / b[0]
__global__ void k_scale_dev(double *__restrict__ y, const double *__restrict__ x, const double *__restrict__ b,
                            int64_t n) {
    const double s = b[0];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = x[i] / s;
}

struct LzWs {
    double *v[3], *ab, *nrm, *part, *T, *theta, *Y;
    void *eig;
    size_t eig_b;
};

LzWs lz_layout(Arena &a, int64_t n, int steps) {
    LzWs s;
    for (int i = 0; i < 3; ++i) s.v[i] = a.take<double>((size_t)n);
    s.ab = a.take<double>(4);
    s.nrm = a.take<double>(1);
    s.part = a.take<double>(std::max(gram_partial_elems(n, 1, 1), colnorm_partial_elems(n, 1)));
    s.T = a.take<double>((size_t)steps * steps);
    s.theta = a.take<double>(steps);
    s.Y = a.take<double>((size_t)steps * steps);
    s.eig_b = eig_ws_bytes(steps);
    s.eig = a.take<char>(s.eig_b);
    return s;
}

unsigned grid_n(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096)); }

}  // namespace

chebdav_status lanczos_ws_bytes(int64_t n, int steps, size_t *bytes) {
    if (steps < 1 || steps > kMaxSteps) return fail(CHEBDAV_EINVAL, "steps must be in [1, %d]", kMaxSteps);
    Arena a;
    a.counting = true;
    (void)lz_layout(a, n, steps);
    *bytes = a.used + 256;
    return CHEBDAV_OK;
}

chebdav_status lanczos_bounds(const Graph *g, int steps, uint64_t seed, double *lower, double *upper,
                              double *alpha_out, double *beta_out, int *steps_done, void *ws, size_t ws_bytes,
                              hipStream_t st) {
    size_t need = 0;
    CD_TRY(lanczos_ws_bytes(g->n, steps, &need));
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "Lanczos workspace too small (%zu < %zu)", ws_bytes, need);
    if (!lower || !upper) return fail(CHEBDAV_EINVAL, "lower/upper are NULL");
    const int64_t n = g->n;
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const LzWs s = lz_layout(a, n, steps);
    double *h = static_cast<double *>(pinned_host(sizeof(double) * (2 + (size_t)steps * steps + steps), 3));
    if (!h) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    double *prev = s.v[0], *cur = s.v[1], *w = s.v[2];
    const unsigned gn = grid_n(n);
    // start vector
    CD_TRY(philox_fill(w, n, 1, 1, seed, kStartColumn, st));
    CD_TRY(colnorms(w, 1, nullptr, 0, nullptr, 1, n, s.nrm, s.part, st));
    hipLaunchKernelGGL(k_scale_dev, dim3(gn), dim3(256), 0, st, cur, w, s.nrm, n);
    CD_LAUNCH_CHECK();
    CD_TRY(fill_f64(prev, n, 0.0, st));
    std::vector<double> al, be;
    double b_prev = 0.0;
    Seg2 vs;
    vs.ld1 = 1;
    vs.p1 = 1;
    for (int j = 0; j < steps; ++j) {
        // w = A v_j - beta_{j-1} v_{j-1}
        CD_TRY((launch_cheb_step<double, double>(g, -1.0, 1.0, -b_prev, cur, 1, prev, 1, w, 1, 1, st)));
        vs.X1 = cur;
        CD_TRY(gram(vs, w, 1, 1, n, s.ab, 1, s.part, st));
        hipLaunchKernelGGL(k_axpy_dev, dim3(gn), dim3(256), 0, st, w, cur, s.ab, n);
        CD_LAUNCH_CHECK();
        CD_TRY(colnorms(w, 1, nullptr, 0, nullptr, 1, n, s.ab + 1, s.part, st));
        CD_HIP(hipMemcpyAsync(h, s.ab, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        const double aj = h[0], bj = h[1];
        if (!std::isfinite(aj) || !std::isfinite(bj)) return fail(CHEBDAV_EBREAKDOWN, "Lanczos produced a non-finite value");
        al.push_back(aj);
        be.push_back(bj);
        if (bj <= 1e-12 * std::max(1.0, std::fabs(aj))) break;
        // v_{j+1} = w / beta_j into the slot of v_{j-1}
        hipLaunchKernelGGL(k_scale_dev, dim3(gn), dim3(256), 0, st, prev, w, s.ab + 1, n);
        CD_LAUNCH_CHECK();
        std::swap(prev, cur);
        b_prev = bj;
    }
    const int k = (int)al.size();
    // T_k and its Ritz values
    double *hT = h + 2;
    for (int i = 0; i < k * k; ++i) hT[i] = 0.0;
    for (int i = 0; i < k; ++i) {
        hT[i * k + i] = al[i];
        if (i + 1 < k) hT[i * k + i + 1] = hT[(i + 1) * k + i] = be[i];
    }
    CD_HIP(hipMemcpyAsync(s.T, hT, sizeof(double) * k * k, hipMemcpyHostToDevice, st));
    CD_TRY(small_eig(s.T, k, k, s.theta, s.Y, k, s.eig, s.eig_b, st));
    double *hth = hT + (size_t)k * k;
    CD_HIP(hipMemcpyAsync(hth, s.theta, sizeof(double) * k, hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    const double bk = be.back();
    *lower = hth[0] - bk;
    *upper = hth[k - 1] + bk;
    for (int i = 0; i < k; ++i) {
        if (alpha_out) alpha_out[i] = al[i];
        if (beta_out) beta_out[i] = be[i];
    }
    if (steps_done) *steps_done = k;
    return CHEBDAV_OK;
}

}  // namespace chebdav
