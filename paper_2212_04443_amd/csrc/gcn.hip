// Learned warm start: a three-layer graph-convolution network whose output
// block seeds the solver's initial vectors (progressive filtering of V_init,
// Alg. 2 steps 2 and 17).  Not part of the paper.
//
//   Z_l = Ahat (H_{l-1} W_l),  H_l = ReLU(Z_l) (l = 1, 2),  X = Z_3,
//   Ahat = D^{-1/2} S D^{-1/2}  (the fused sparse step with alpha = 1, beta = gamma = 0)
//
// Backward, with G_l = Ahat dZ_l (Ahat is symmetric):
//   dW_l = H_{l-1}^T G_l,  dH_{l-1} = G_l W_l^T,  dZ_{l-1} = dH_{l-1} .* [H_{l-1} > 0].
//
// Training loss (rotation and sign invariant): with targets U (n x k,
// orthonormal), G = X^T X and M = X^T U,
//   L = 1 - tr(U^T X G^{-1} X^T U) / k,
//   dL/dX = X A + U B,  A = (2/k) G^{-1} M M^T G^{-1},  B = -(2/k) M^T G^{-1}.
//
// All network arithmetic is FP32; the loss and its small matrices are FP64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kT = 64;   // output tile edge
constexpr int kKc = 16;  // reduction chunk

// C (n x q) = A (n x p) * op(B), op(B) = B (p x q, ldb) or B^T (B is q x p, ldb).
template <bool TRANS_B>
__global__ void __launch_bounds__(256) k_sgemm_nn(const float *__restrict__ A, int64_t lda, const float *__restrict__ B,
                                                  int64_t ldb, float *__restrict__ C, int64_t ldc, int64_t n, int p,
                                                  int q) {
    __shared__ float sa[kT][kKc + 1];
    __shared__ float sb[kKc][kT + 1];
    const int64_t r0 = (int64_t)blockIdx.x * kT;
    const int j0 = blockIdx.y * kT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < p; k0 += kKc) {
        for (int e = threadIdx.x; e < kT * kKc; e += 256) {
            const int rr = e / kKc, kk = e % kKc;
            const int64_t row = r0 + rr;
            sa[rr][kk] = (row < n && k0 + kk < p) ? A[row * lda + k0 + kk] : 0.f;
            const int kb = e / kT, c = e % kT;
            float bv = 0.f;
            if (k0 + kb < p && j0 + c < q)
                bv = TRANS_B ? B[(int64_t)(j0 + c) * ldb + k0 + kb] : B[(int64_t)(k0 + kb) * ldb + j0 + c];
            sb[kb][c] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKc; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sa[ty * 4 + u][kk];
                b[u] = sb[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t row = r0 + ty * 4 + u;
        if (row >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j < q) C[row * ldc + j] = acc[u][v];
        }
    }
}

// Partial C = A^T B over row splits (A: n x p, B: n x q), FP32 products summed in FP32
// within a split; the splits are then added in a fixed order in FP64.
__global__ void __launch_bounds__(256) k_sgemm_tn(const float *__restrict__ A, int64_t lda, const float *__restrict__ B,
                                                  int64_t ldb, int64_t n, int p, int q, int64_t rows_per_split,
                                                  double *__restrict__ part) {
    __shared__ float sa[kKc][kT + 1];
    __shared__ float sb[kKc][kT + 1];
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int64_t r_beg = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r_end = min(n, r_beg + rows_per_split);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    float acc[4][4] = {};
    for (int64_t r0 = r_beg; r0 < r_end; r0 += kKc) {
        for (int e = threadIdx.x; e < kKc * kT; e += 256) {
            const int kk = e / kT, c = e % kT;
            const int64_t row = r0 + kk;
            const bool rv = row < r_end;
            sa[kk][c] = (rv && i0 + c < p) ? A[row * lda + i0 + c] : 0.f;
            sb[kk][c] = (rv && j0 + c < q) ? B[row * ldb + j0 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKc; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sa[kk][ty * 4 + u];
                b[u] = sb[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    double *out = part + (int64_t)blockIdx.z * p * q;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
            if (i < p && j < q) out[(int64_t)i * q + j] = (double)acc[u][v];
        }
}

__global__ void k_reduce_to_f32(const double *__restrict__ part, int splits, int64_t E, float *__restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * E + e];
    C[e] = (float)s;
}

__global__ void k_relu(float *__restrict__ X, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) X[e] = fmaxf(X[e], 0.f);
}

// dZ = dH .* [H > 0], in place on dH.
__global__ void k_relu_mask(float *__restrict__ dH, const float *__restrict__ H, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride)
        if (!(H[e] > 0.f)) dH[e] = 0.f;
}

// Input features: n_gauss standard normal channels (Box-Muller on Philox4x32-10
// counters (row, row >> 32, pair, 1), key = seed) and sqrt(deg / mean deg).
__global__ void k_features(const int32_t *__restrict__ deg, double inv_mean_deg, int64_t n, int n_gauss, uint64_t seed,
                           float *__restrict__ X, int64_t ldx) {
    const int pairs = (n_gauss + 1) / 2;
    const int64_t total = n * (int64_t)(pairs + 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t r = e / (pairs + 1);
        const int pr = (int)(e - r * (pairs + 1));
        if (pr == pairs) {
            X[r * ldx + n_gauss] = (float)sqrt((double)deg[r] * inv_mean_deg);
            continue;
        }
        uint32_t c[4] = {(uint32_t)r, (uint32_t)((uint64_t)r >> 32), (uint32_t)pr, 1u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = ((double)(c[0] >> 8) + 0.5) * 0x1.0p-24;  // (0, 1)
        const double u2 = (double)(c[1] >> 8) * 0x1.0p-24;          // [0, 1)
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586 * u2;
        X[r * ldx + 2 * pr] = (float)(rad * cos(ang));
        if (2 * pr + 1 < n_gauss) X[r * ldx + 2 * pr + 1] = (float)(rad * sin(ang));
    }
}


// Loss and gradient coefficients from G = X^T X (kx x kx) and M = X^T U (kx x ku),
// one workgroup: Cholesky of G, Ginv, L = 1 - tr(M^T Ginv M)/ku,
// A = (2/ku) Ginv M M^T Ginv (kx x kx), B = -(2/ku) M^T Ginv (ku x kx).
constexpr int kMaxK = 64;
__global__ void __launch_bounds__(256) k_loss_coeffs(const double *__restrict__ G, const double *__restrict__ M,
                                                     int kx, int ku, double *__restrict__ Acoef,
                                                     double *__restrict__ Bc, double *__restrict__ loss,
                                                     int *__restrict__ bad) {
    __shared__ double L[kMaxK][kMaxK + 1];   // Cholesky factor (lower)
    __shared__ double Gi[kMaxK][kMaxK + 1];  // G^{-1}
    __shared__ double P[kMaxK][kMaxK + 1];   // Ginv M
    __shared__ double red[256];
    const int tid = threadIdx.x;
    for (int e = tid; e < kx * kx; e += blockDim.x) L[e / kx][e % kx] = G[e];
    __syncthreads();
    if (tid == 0) {
        int b = 0;
        for (int k = 0; k < kx; ++k) {
            double d = L[k][k];
            for (int j = 0; j < k; ++j) d -= L[k][j] * L[k][j];
            if (!(d > 0.0)) {
                b = 1;
                d = 1e-300;
            }
            L[k][k] = sqrt(d);
            for (int i = k + 1; i < kx; ++i) {
                double s = L[i][k];
                for (int j = 0; j < k; ++j) s -= L[i][j] * L[k][j];
                L[i][k] = s / L[k][k];
            }
        }
        *bad = b;
    }
    __syncthreads();
    // Ginv column by column: solve L y = e_j, L^T x = y
    if (tid < kx) {
        const int j = tid;
        double y[kMaxK];
        for (int i = 0; i < kx; ++i) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int l = 0; l < i; ++l) s -= L[i][l] * y[l];
            y[i] = s / L[i][i];
        }
        for (int i = kx - 1; i >= 0; --i) {
            double s = y[i];
            for (int l = i + 1; l < kx; ++l) s -= L[l][i] * Gi[l][j];
            Gi[i][j] = s / L[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < kx * ku; e += blockDim.x) {
        const int i = e / ku, c = e % ku;
        double s = 0.0;
        for (int l = 0; l < kx; ++l) s += Gi[i][l] * M[l * ku + c];
        P[i][c] = s;
        Bc[c * kx + i] = -2.0 / ku * s;
    }
    __syncthreads();
    // tr(M^T Ginv M) = sum_ic M[i][c] P[i][c]
    double part = 0.0;
    for (int e = tid; e < kx * ku; e += blockDim.x) part += M[e] * P[e / ku][e % ku];
    red[tid] = part;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        *loss = 1.0 - t / ku;
    }
    // A = (2/ku) P P^T
    for (int e = tid; e < kx * kx; e += blockDim.x) {
        const int i = e / kx, j = e % kx;
        double s = 0.0;
        for (int c = 0; c < ku; ++c) s += P[i][c] * P[j][c];
        Acoef[e] = 2.0 / ku * s;
    }
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t count, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned grid1(int64_t total) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 8192));
}

int tn_splits(int64_t n, int p, int q) {
    const int tiles = (int)(ceil_div(p, kT) * ceil_div(q, kT));
    int64_t s = std::max<int64_t>(1, 512 / tiles);
    s = std::min<int64_t>(s, std::max<int64_t>(1, ceil_div(n, 1024)));
    return (int)s;
}

}  // namespace

// ---- building blocks -------------------------------------------------------
chebdav_status sgemm_nn(const float *A, int64_t lda, const float *B, int64_t ldb, bool transB, float *C,
                        int64_t ldc, int64_t n, int p, int q, hipStream_t st) {
    if (n == 0 || q == 0) return CHEBDAV_OK;
    const dim3 grid((unsigned)ceil_div(n, kT), (unsigned)ceil_div(q, kT));
    if (transB)
        hipLaunchKernelGGL(k_sgemm_nn<true>, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, n, p, q);
    else
        hipLaunchKernelGGL(k_sgemm_nn<false>, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, n, p, q);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

size_t sgemm_tn_partial_elems(int64_t n, int p, int q) { return (size_t)tn_splits(n, p, q) * p * q; }

chebdav_status sgemm_tn(const float *A, int64_t lda, const float *B, int64_t ldb, int64_t n, int p, int q, float *C,
                        double *part, hipStream_t st) {
    const int splits = tn_splits(n, p, q);
    const int64_t rps = ceil_div(ceil_div(n, splits), kKc) * kKc;
    const dim3 grid((unsigned)ceil_div(p, kT), (unsigned)ceil_div(q, kT), (unsigned)splits);
    hipLaunchKernelGGL(k_sgemm_tn, grid, dim3(256), 0, st, A, lda, B, ldb, n, p, q, rps, part);
    CD_LAUNCH_CHECK();
    const int64_t E = (int64_t)p * q;
    hipLaunchKernelGGL(k_reduce_to_f32, dim3((unsigned)ceil_div(E, 256)), dim3(256), 0, st, part, splits, E, C);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

// ---- network ----------------------------------------------------------------
struct GcnWs {
    float *P, *G, *dH;
    double *part;
};

static GcnWs gcn_layout(Arena &a, int64_t n, const int dims[4]) {
    const int wmax = std::max(std::max(dims[0], dims[1]), std::max(dims[2], dims[3]));
    GcnWs s;
    s.P = a.take<float>((size_t)n * wmax);
    s.G = a.take<float>((size_t)n * wmax);
    s.dH = a.take<float>((size_t)n * wmax);
    size_t pe = 0;
    for (int l = 0; l < 3; ++l) pe = std::max(pe, sgemm_tn_partial_elems(n, dims[l], dims[l + 1]));
    s.part = a.take<double>(pe);
    return s;
}

size_t gcn_ws_bytes(int64_t n, const int dims[4]) {
    Arena a;
    a.counting = true;
    (void)gcn_layout(a, n, dims);
    return a.used + 256;
}

static chebdav_status check_dims(const int dims[4]) {
    for (int l = 0; l < 4; ++l)
        if (dims[l] < 1 || dims[l] > 256) return fail(CHEBDAV_EINVAL, "GCN widths must be in [1, 256]");
    return CHEBDAV_OK;
}

chebdav_status gcn_forward(const Graph *g, const int dims[4], const float *X0, const float *const W[3], float *acts,
                           float *out, void *ws, size_t ws_bytes, hipStream_t st) {
    CD_TRY(check_dims(dims));
    const int64_t n = g->n;
    if (!ws || ws_bytes < gcn_ws_bytes(n, dims)) return fail(CHEBDAV_ENOMEM, "GCN workspace too small");
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const GcnWs s = gcn_layout(a, n, dims);
    float *H1 = acts, *H2 = acts + (size_t)n * dims[1];
    const float *Hin = X0;
    for (int l = 0; l < 3; ++l) {
        const int p = dims[l], q = dims[l + 1];
        CD_TRY(sgemm_nn(Hin, p, W[l], q, false, s.P, q, n, p, q, st));
        float *Z = l == 0 ? H1 : (l == 1 ? H2 : out);
        CD_TRY((launch_cheb_step<float, float>(g, 1.0, 0.0, 0.0, s.P, q, nullptr, 0, Z, q, q, st)));
        if (l < 2) {
            hipLaunchKernelGGL(k_relu, dim3(grid1(n * q)), dim3(256), 0, st, Z, n * (int64_t)q);
            CD_LAUNCH_CHECK();
        }
        Hin = Z;
    }
    return CHEBDAV_OK;
}

chebdav_status gcn_backward(const Graph *g, const int dims[4], const float *X0, const float *const W[3],
                            const float *acts, const float *d_out, float *const dW[3], void *ws, size_t ws_bytes,
                            hipStream_t st) {
    CD_TRY(check_dims(dims));
    const int64_t n = g->n;
    if (!ws || ws_bytes < gcn_ws_bytes(n, dims)) return fail(CHEBDAV_ENOMEM, "GCN workspace too small");
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const GcnWs s = gcn_layout(a, n, dims);
    const float *H[3] = {X0, acts, acts + (size_t)n * dims[1]};
    const float *dZ = d_out;
    for (int l = 2; l >= 0; --l) {
        const int p = dims[l], q = dims[l + 1];
        // G = Ahat dZ
        CD_TRY((launch_cheb_step<float, float>(g, 1.0, 0.0, 0.0, dZ, q, nullptr, 0, s.G, q, q, st)));
        // dW = H_{l-1}^T G
        CD_TRY(sgemm_tn(H[l], p, s.G, q, n, p, q, dW[l], s.part, st));
        if (l > 0) {
            // dH = G W^T, then mask with the ReLU of layer l-1
            CD_TRY(sgemm_nn(s.G, q, W[l], q, true, s.dH, p, n, q, p, st));
            hipLaunchKernelGGL(k_relu_mask, dim3(grid1(n * p)), dim3(256), 0, st, s.dH, H[l], n * (int64_t)p);
            CD_LAUNCH_CHECK();
            dZ = s.dH;
        }
    }
    return CHEBDAV_OK;
}

chebdav_status gcn_features(const Graph *g, uint64_t seed, int n_gauss, float *X, int64_t ldx, hipStream_t st) {
    if (n_gauss < 0 || ldx < n_gauss + 1) return fail(CHEBDAV_EINVAL, "bad feature width");
    if (!X) return fail(CHEBDAV_EINVAL, "X is NULL");
    // the degrees sum to the stored nonzeros, which the graph keeps on the host
    const double mean = g->nnz > 0 ? (double)g->nnz / (double)g->n : 1.0;
    const int pairs = (n_gauss + 1) / 2;
    hipLaunchKernelGGL(k_features, dim3(grid1(g->n * (pairs + 1))), dim3(256), 0, st, g->deg, 1.0 / mean, g->n,
                       n_gauss, seed, X, ldx);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

// ---- loss -------------------------------------------------------------------
struct LossWs {
    double *X64, *dX64, *G, *M, *A, *B, *part, *loss;
    int *bad;
};

static LossWs loss_layout(Arena &a, int64_t n, int kx, int ku) {
    LossWs s;
    s.X64 = a.take<double>((size_t)n * kx);
    s.dX64 = a.take<double>((size_t)n * kx);
    s.G = a.take<double>((size_t)kx * kx);
    s.M = a.take<double>((size_t)kx * ku);
    s.A = a.take<double>((size_t)kx * kx);
    s.B = a.take<double>((size_t)kx * ku);
    s.part = a.take<double>(std::max(gram_partial_elems(n, kx, kx), gram_partial_elems(n, kx, ku)));
    s.loss = a.take<double>(2);
    s.bad = a.take<int>(2);
    return s;
}

size_t loss_ws_bytes(int64_t n, int kx, int ku) {
    Arena a;
    a.counting = true;
    (void)loss_layout(a, n, kx, ku);
    return a.used + 256;
}

void *pinned_host(size_t bytes, int slot);

chebdav_status subspace_loss(const float *X, int64_t ldx, const double *U, int64_t ldu, int64_t n, int kx, int ku,
                             double *loss_host, float *dX, int64_t lddx, void *ws, size_t ws_bytes, hipStream_t st) {
    if (kx < 1 || kx > kMaxK || ku < 1 || ku > kMaxK) return fail(CHEBDAV_EUNSUPPORTED, "loss widths must be in [1, 64]");
    if (n < kx) return fail(CHEBDAV_EINVAL, "n < kx");
    if (!ws || ws_bytes < loss_ws_bytes(n, kx, ku)) return fail(CHEBDAV_ENOMEM, "loss workspace too small");
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const LossWs s = loss_layout(a, n, kx, ku);
    CD_TRY((copy_block<float, double>(X, ldx, s.X64, kx, kx, n, st)));
    Seg2 xs;
    xs.X1 = s.X64;
    xs.ld1 = kx;
    xs.p1 = kx;
    CD_TRY(gram(xs, s.X64, kx, kx, n, s.G, kx, s.part, st));
    CD_TRY(gram(xs, U, ldu, ku, n, s.M, ku, s.part, st));
    hipLaunchKernelGGL(k_loss_coeffs, dim3(1), dim3(256), 0, st, s.G, s.M, kx, ku, s.A, s.B, s.loss, s.bad);
    CD_LAUNCH_CHECK();
    if (dX) {
        // dX = X A + U B
        CD_TRY(update(xs, s.A, kx, 1.0, 0.0, s.dX64, kx, kx, n, st));
        Seg2 us;
        us.X1 = U;
        us.ld1 = ldu;
        us.p1 = ku;
        CD_TRY(update(us, s.B, kx, 1.0, 1.0, s.dX64, kx, kx, n, st));
        CD_TRY((copy_block<double, float>(s.dX64, kx, dX, lddx, kx, n, st)));
    }
    double *h = static_cast<double *>(pinned_host(2 * sizeof(double), 3));
    if (!h) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    CD_HIP(hipMemcpyAsync(h, s.loss, sizeof(double), hipMemcpyDeviceToHost, st));
    CD_HIP(hipMemcpyAsync(h + 1, s.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    CD_HIP(hipStreamSynchronize(st));
    int bad = 0;
    memcpy(&bad, h + 1, sizeof(int));
    if (bad) return fail(CHEBDAV_EBREAKDOWN, "X^T X is not positive definite (rank-deficient network output)");
    if (loss_host) *loss_host = h[0];
    return CHEBDAV_OK;
}

chebdav_status adam_step(float *w, const float *g, float *m, float *v, int64_t count, double lr, double b1,
                         double b2, double eps, int step, hipStream_t st) {
    if (step < 1 || count < 0) return fail(CHEBDAV_EINVAL, "bad Adam arguments");
    if (count == 0) return CHEBDAV_OK;
    const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st, w, g, m, v, count, (float)lr,
                       (float)b1, (float)b2, (float)eps, c1, c2);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

// ---- Rayleigh-Ritz of a block: the warm-start vectors -------------------------
struct RrWs {
    double *Q, *W, *H, *Y, *part;
    void *orth, *eig;
    size_t orth_b, eig_b;
};

static RrWs rr_layout(Arena &a, int64_t n, int k) {
    RrWs s;
    s.Q = a.take<double>((size_t)n * k);
    s.W = a.take<double>((size_t)n * k);
    s.H = a.take<double>((size_t)k * k);
    s.Y = a.take<double>((size_t)k * k);
    s.part = a.take<double>(gram_partial_elems(n, k, k));
    s.orth_b = orth_ws_bytes(n, 0, k);
    s.orth = a.take<char>(s.orth_b);
    s.eig_b = eig_ws_bytes(k);
    s.eig = a.take<char>(s.eig_b);
    return s;
}

size_t rr_ws_bytes(int64_t n, int k) {
    Arena a;
    a.counting = true;
    (void)rr_layout(a, n, k);
    return a.used + 256;
}

// V (n x k, ldv) = Ritz vectors of span(X) for A, in ascending order of their
// Rayleigh quotients (written to ritz[k]); X is orthonormalized first (random
// replacement of dependent columns, Philox key = seed).
chebdav_status rayleigh_ritz(const Graph *g, const float *X, int64_t ldx, int k, uint64_t seed, double *V,
                             int64_t ldv, double *ritz, void *ws, size_t ws_bytes, hipStream_t st) {
    const int64_t n = g->n;
    if (k < 1 || k > update_max_inplace_cols()) return fail(CHEBDAV_EUNSUPPORTED, "k must be in [1, 64]");
    if (!ws || ws_bytes < rr_ws_bytes(n, k)) return fail(CHEBDAV_ENOMEM, "Rayleigh-Ritz workspace too small");
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const RrWs s = rr_layout(a, n, k);
    CD_TRY((copy_block<float, double>(X, ldx, s.Q, k, k, n, st)));
    Seg2 none;
    uint64_t next = 0;
    int rep = 0;
    CD_TRY(orthonormalize(none, s.Q, k, k, n, seed, &next, &rep, s.orth, s.orth_b, st));
    CD_TRY((launch_cheb_step<double, double>(g, -1.0, 1.0, 0.0, s.Q, k, nullptr, 0, s.W, k, k, st)));
    Seg2 qs;
    qs.X1 = s.Q;
    qs.ld1 = k;
    qs.p1 = k;
    CD_TRY(gram(qs, s.W, k, k, n, s.H, k, s.part, st));
    CD_TRY(small_eig(s.H, k, k, ritz, s.Y, k, s.eig, s.eig_b, st));
    CD_TRY(update(qs, s.Y, k, 1.0, 0.0, V, ldv, k, n, st));
    return CHEBDAV_OK;
}

}  // namespace chebdav
