// Symmetric eigendecomposition H = Y diag(w) Y^T of the small Rayleigh-quotient
// matrix (Alg. 2 step 9), ascending.  Pipeline:
//   1. Householder tridiagonalization Q^T H Q = T (one workgroup; H stays in
//      L2, the current Householder vector in LDS);
//   2. eigenvalues of T by bisection on Sturm counts, one thread per eigenvalue;
//   3. eigenvectors of T by inverse iteration with the LU factorization (with
//      partial pivoting) of T - w I, one thread per eigenvector, factors stored
//      interleaved across threads so every access is coalesced;
//   4. modified Gram-Schmidt inside tight clusters (gap <= 1e-6 ||T||);
//   5. back-transformation Y = Q Z, one wavefront per eigenvector;
//   6. two Newton-Schulz steps Y <- Y (3 I - Y^T Y)/2 restore orthogonality to
//      rounding level (inverse-iteration vectors of distinct eigenvalues are
//      orthogonal only to about eps ||T|| / gap).
#include <cfloat>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kMaxN = 1024;
constexpr double kEps = DBL_EPSILON * 0.5;
constexpr double kTightRel = 1e-6;

struct EigWs {
    double *A, *Vh, *Zv, *dl, *dd, *du, *du2, *x;
    int *ipiv;
    double *d, *e, *tau, *w, *par, *G, *Bm, *T, *part;
};

EigWs eig_layout(Arena &a, int n) {
    EigWs s;
    const size_t nn = (size_t)n * n;
    s.A = a.take<double>(nn);
    s.Vh = a.take<double>(nn);
    s.Zv = a.take<double>(nn);
    s.dl = a.take<double>(nn);
    s.dd = a.take<double>(nn);
    s.du = a.take<double>(nn);
    s.du2 = a.take<double>(nn);
    s.x = a.take<double>(nn);
    s.ipiv = a.take<int>(nn);
    s.d = a.take<double>(n);
    s.e = a.take<double>(n);
    s.tau = a.take<double>(n);
    s.w = a.take<double>(n);
    s.par = a.take<double>(4);
    s.G = a.take<double>(nn);
    s.Bm = a.take<double>(nn);
    s.T = a.take<double>(nn);
    s.part = a.take<double>(gram_partial_elems(n, n, n));
    return s;
}

__global__ void __launch_bounds__(1024) k_tridiag(const double *__restrict__ H, int64_t ldh, int n,
                                                  double *__restrict__ A, double *__restrict__ Vh,
                                                  double *__restrict__ d, double *__restrict__ e,
                                                  double *__restrict__ tau) {
    __shared__ double v[kMaxN];
    __shared__ double wsh[kMaxN];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = lane_id(), wv = tid / kWave, nw = nt / kWave;
    for (int q = tid; q < n * n; q += nt) A[q] = H[(int64_t)(q / n) * ldh + (q % n)];
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        for (int i = tid; i < m; i += nt) v[i] = A[(k + 1 + i) * n + k];
        __syncthreads();
        double part = 0.0;
        for (int i = 1 + tid; i < m; i += nt) part += v[i] * v[i];
        const double ss = block_sum(part);
        const double x0 = v[0];
        if (ss == 0.0) {
            if (tid == 0) {
                tau[k] = 0.0;
                e[k] = x0;
                d[k] = A[k * n + k];
            }
            for (int i = tid; i < m; i += nt) Vh[k * n + i] = 0.0;
            __syncthreads();
            continue;
        }
        const double alpha = -copysign(sqrt(x0 * x0 + ss), x0);
        const double v0 = x0 - alpha;
        const double t = 2.0 / (v0 * v0 + ss);
        __syncthreads();
        if (tid == 0) {
            v[0] = v0;
            tau[k] = t;
            e[k] = alpha;
            d[k] = A[k * n + k];
        }
        __syncthreads();
        for (int i = wv; i < m; i += nw) {
            const double *row = A + (k + 1 + i) * n + (k + 1);
            double s = 0.0;
            for (int j = lane; j < m; j += kWave) s += row[j] * v[j];
            s = wave_sum(s);
            if (lane == 0) wsh[i] = t * s;
        }
        __syncthreads();
        part = 0.0;
        for (int i = tid; i < m; i += nt) part += wsh[i] * v[i];
        const double K = 0.5 * t * block_sum(part);
        for (int i = tid; i < m; i += nt) wsh[i] -= K * v[i];
        __syncthreads();
        for (int q = tid; q < m * m; q += nt) {
            const int i = q / m, j = q % m;
            A[(k + 1 + i) * n + (k + 1 + j)] -= v[i] * wsh[j] + wsh[i] * v[j];
        }
        for (int i = tid; i < m; i += nt) Vh[k * n + i] = v[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            d[n - 2] = A[(n - 2) * n + (n - 2)];
            e[n - 2] = A[(n - 1) * n + (n - 2)];
            d[n - 1] = A[(n - 1) * n + (n - 1)];
        } else {
            d[0] = A[0];
        }
        e[n - 1] = 0.0;
    }
}

__device__ inline void gersh(const double *d, const double *e, int n, double &gl, double &gu,
                             double &emax2) {
    gl = DBL_MAX;
    gu = -DBL_MAX;
    emax2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
        const double er = i + 1 < n ? fabs(e[i]) : 0.0;
        gl = fmin(gl, d[i] - el - er);
        gu = fmax(gu, d[i] + el + er);
        emax2 = fmax(emax2, er * er);
    }
}

// Number of eigenvalues of T smaller than x (Sturm sequence).
__device__ inline int sturm(const double *d, const double *e, int n, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

__global__ void k_bisect(const double *__restrict__ d, const double *__restrict__ e, int n,
                         double *__restrict__ w, double *__restrict__ par) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double gl, gu, emax2;
    gersh(d, e, n, gl, gu, emax2);
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double atol = 2.0 * kEps * tnorm + pivmin;
    double lo = gl - atol - 2.0 * kEps * tnorm, hi = gu + atol + 2.0 * kEps * tnorm;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (hi - lo <= atol || mid <= lo || mid >= hi) break;
        if (sturm(d, e, n, mid, pivmin) > j)
            hi = mid;
        else
            lo = mid;
    }
    w[j] = 0.5 * (lo + hi);
    if (j == 0) {
        par[0] = tnorm;
        par[1] = pivmin;
    }
}

__device__ inline double hash_unit(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// Inverse iteration, one thread per eigenvector; arrays interleaved as a[i*n + j].
__global__ void k_inviter(const double *__restrict__ d, const double *__restrict__ e, int n,
                          const double *__restrict__ w, const double *__restrict__ par,
                          double *__restrict__ dl, double *__restrict__ dd, double *__restrict__ du,
                          double *__restrict__ du2, double *__restrict__ x, int *__restrict__ ipiv,
                          double *__restrict__ Zv) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double tnorm = par[0];
    const double tight = kTightRel * tnorm;
    const double pert = 10.0 * kEps * fmax(tnorm, DBL_MIN);
    int pos = 0;
    for (int i = j - 1; i >= 0 && w[i + 1] - w[i] <= tight; --i) ++pos;
    const double lam = w[j] + pert * pos;
    const double tiny = kEps * fmax(tnorm, DBL_MIN);
#define IX(i) ((int64_t)(i) * n + j)
    if (n == 1) {
        Zv[0] = 1.0;
        return;
    }
    for (int i = 0; i < n; ++i) dd[IX(i)] = d[i] - lam;
    for (int i = 0; i + 1 < n; ++i) {
        dl[IX(i)] = e[i];
        du[IX(i)] = e[i];
    }
    for (int i = 0; i + 2 < n; ++i) du2[IX(i)] = 0.0;
    // LU with partial pivoting of the tridiagonal T - lam I
    for (int i = 0; i + 1 < n; ++i) {
        const double a = dd[IX(i)], b = dl[IX(i)];
        if (fabs(a) >= fabs(b)) {
            ipiv[IX(i)] = i;
            const double piv = a != 0.0 ? a : tiny;
            dd[IX(i)] = piv;
            const double f = b / piv;
            dl[IX(i)] = f;
            dd[IX(i + 1)] -= f * du[IX(i)];
        } else {
            ipiv[IX(i)] = i + 1;
            const double f = a / b;
            dd[IX(i)] = b;
            dl[IX(i)] = f;
            const double tmp = du[IX(i)];
            du[IX(i)] = dd[IX(i + 1)];
            dd[IX(i + 1)] = tmp - f * dd[IX(i + 1)];
            if (i + 2 < n) {
                du2[IX(i)] = du[IX(i + 1)];
                du[IX(i + 1)] = -f * du[IX(i + 1)];
            }
        }
    }
    if (dd[IX(n - 1)] == 0.0) dd[IX(n - 1)] = tiny;
    for (int i = 0; i < n; ++i) x[IX(i)] = hash_unit((uint32_t)i, (uint32_t)j);
    for (int it = 0; it < 3; ++it) {
        // forward: apply the row interchanges and L
        for (int i = 0; i + 1 < n; ++i) {
            const double f = dl[IX(i)];
            if (ipiv[IX(i)] == i) {
                x[IX(i + 1)] -= f * x[IX(i)];
            } else {
                const double t0 = x[IX(i)];
                x[IX(i)] = x[IX(i + 1)];
                x[IX(i + 1)] = t0 - f * x[IX(i)];
            }
        }
        // back substitution with U (diagonal dd, super-diagonals du, du2)
        x[IX(n - 1)] /= dd[IX(n - 1)];
        x[IX(n - 2)] = (x[IX(n - 2)] - du[IX(n - 2)] * x[IX(n - 1)]) / dd[IX(n - 2)];
        for (int i = n - 3; i >= 0; --i)
            x[IX(i)] = (x[IX(i)] - du[IX(i)] * x[IX(i + 1)] - du2[IX(i)] * x[IX(i + 2)]) / dd[IX(i)];
        double mx = 0.0;
        for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(x[IX(i)]));
        const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
        double s2 = 0.0;
        for (int i = 0; i < n; ++i) {
            const double v = x[IX(i)] * sc;
            s2 += v * v;
        }
        const double nr = sc / sqrt(s2);
        for (int i = 0; i < n; ++i) x[IX(i)] *= nr;
    }
    for (int i = 0; i < n; ++i) Zv[(int64_t)j * n + i] = x[IX(i)];
#undef IX
}

// Modified Gram-Schmidt (two passes) inside clusters with gaps below the tight threshold.
__global__ void __launch_bounds__(256) k_cluster_mgs(const double *__restrict__ w,
                                                     const double *__restrict__ par, int n,
                                                     double *__restrict__ Zv) {
    const int j = blockIdx.x;
    const double tight = kTightRel * par[0];
    if (!(j == 0 || w[j] - w[j - 1] > tight)) return;
    if (j + 1 >= n || w[j + 1] - w[j] > tight) return;
    int end = j + 1;
    while (end < n && w[end] - w[end - 1] <= tight) ++end;
    for (int c = j + 1; c < end; ++c) {
        double *zc = Zv + (int64_t)c * n;
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = j; i < c; ++i) {
                const double *zi = Zv + (int64_t)i * n;
                double part = 0.0;
                for (int k = threadIdx.x; k < n; k += blockDim.x) part += zi[k] * zc[k];
                const double dot = block_sum(part);
                for (int k = threadIdx.x; k < n; k += blockDim.x) zc[k] -= dot * zi[k];
                __syncthreads();
            }
        }
        double part = 0.0;
        for (int k = threadIdx.x; k < n; k += blockDim.x) part += zc[k] * zc[k];
        const double nr = sqrt(block_sum(part));
        for (int k = threadIdx.x; k < n; k += blockDim.x) zc[k] /= nr;
        __syncthreads();
    }
}

// Y(:, j) = Q z_j with Q = H_0 H_1 ... H_{n-3}; one wavefront per eigenvector.
constexpr int kTpl = kMaxN / kWave;
__global__ void __launch_bounds__(256) k_backtransform(const double *__restrict__ Vh,
                                                       const double *__restrict__ tau,
                                                       const double *__restrict__ Zv, int n,
                                                       double *__restrict__ Y, int64_t ldy) {
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= n) return;
    const int lane = lane_id();
    const int tpl = (n + kWave - 1) / kWave;
    double z[kTpl];
#pragma unroll
    for (int t = 0; t < kTpl; ++t) {
        const int i = lane + t * kWave;
        z[t] = (t < tpl && i < n) ? Zv[(int64_t)j * n + i] : 0.0;
    }
    for (int k = n - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const double *vk = Vh + (int64_t)k * n - (k + 1);  // vk[i] for i in [k+1, n)
        double dot = 0.0;
#pragma unroll
        for (int t = 0; t < kTpl; ++t) {
            const int i = lane + t * kWave;
            if (t < tpl && i > k && i < n) dot += vk[i] * z[t];
        }
        const double s = tk * wave_sum(dot);
#pragma unroll
        for (int t = 0; t < kTpl; ++t) {
            const int i = lane + t * kWave;
            if (t < tpl && i > k && i < n) z[t] -= s * vk[i];
        }
    }
#pragma unroll
    for (int t = 0; t < kTpl; ++t) {
        const int i = lane + t * kWave;
        if (t < tpl && i < n) Y[(int64_t)i * ldy + j] = z[t];
    }
}

__global__ void k_ns_prep(const double *__restrict__ G, int n, double *__restrict__ B) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)n * n) return;
    const int i = (int)(q / n), j = (int)(q % n);
    B[q] = (i == j ? 1.5 : 0.0) - 0.5 * G[q];
}

__global__ void k_copy_vec(const double *__restrict__ s, double *__restrict__ d, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

}  // namespace

size_t eig_ws_bytes(int n) {
    Arena a;
    a.counting = true;
    (void)eig_layout(a, n);
    return a.used + 256;
}

chebdav_status small_eig(const double *H, int64_t ldh, int n, double *evals, double *Y,
                         int64_t ldy, void *ws, size_t ws_bytes, hipStream_t st) {
    if (n < 1 || n > kMaxN) return fail(CHEBDAV_EUNSUPPORTED, "eigenproblem size %d outside [1, %d]", n, kMaxN);
    if (ldh < n || ldy < n) return fail(CHEBDAV_EINVAL, "leading dimension < n");
    const size_t need = eig_ws_bytes(n);
    if (ws_bytes < need) return fail(CHEBDAV_ENOMEM, "eig workspace too small (%zu < %zu)", ws_bytes, need);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    EigWs s = eig_layout(a, n);
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(1024), 0, st, H, ldh, n, s.A, s.Vh, s.d, s.e, s.tau);
    CD_LAUNCH_CHECK();
    const unsigned g64 = (unsigned)ceil_div(n, 64);
    hipLaunchKernelGGL(k_bisect, dim3(g64), dim3(64), 0, st, s.d, s.e, n, s.w, s.par);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_inviter, dim3(g64), dim3(64), 0, st, s.d, s.e, n, s.w, s.par, s.dl, s.dd,
                       s.du, s.du2, s.x, s.ipiv, s.Zv);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cluster_mgs, dim3(n), dim3(256), 0, st, s.w, s.par, n, s.Zv);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_backtransform, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, s.Vh, s.tau,
                       s.Zv, n, Y, ldy);
    CD_LAUNCH_CHECK();
    // two Newton-Schulz steps: T = Y B1, Y = T B2
    const unsigned gnn = (unsigned)ceil_div((int64_t)n * n, 256);
    {
        Seg2 sy;
        sy.X1 = Y;
        sy.ld1 = ldy;
        sy.p1 = n;
        CD_TRY(gram(sy, Y, ldy, n, n, s.G, n, s.part, st));
        hipLaunchKernelGGL(k_ns_prep, dim3(gnn), dim3(256), 0, st, s.G, n, s.Bm);
        CD_LAUNCH_CHECK();
        CD_TRY(update(sy, s.Bm, n, 1.0, 0.0, s.T, n, n, n, st));
    }
    {
        Seg2 stt;
        stt.X1 = s.T;
        stt.ld1 = n;
        stt.p1 = n;
        CD_TRY(gram(stt, s.T, n, n, n, s.G, n, s.part, st));
        hipLaunchKernelGGL(k_ns_prep, dim3(gnn), dim3(256), 0, st, s.G, n, s.Bm);
        CD_LAUNCH_CHECK();
        CD_TRY(update(stt, s.Bm, n, 1.0, 0.0, Y, ldy, n, n, st));
    }
    hipLaunchKernelGGL(k_copy_vec, dim3(g64), dim3(64), 0, st, s.w, evals, n);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
