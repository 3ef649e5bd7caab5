// One-workgroup kernels on small (kb x kb or k x k) matrices.
#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kMaxKb = 64;

// Cholesky factor and inverse for Cholesky QR.  One workgroup of 256 threads on
// a 16 x 16 grid; thread (ti, tj) owns the entries (ti + 16 a, tj + 16 b) of the
// kb x kb working matrix in LDS, so every step updates all entries in parallel
// without index arithmetic.  Two barriers per step: the diagonal of R is kept
// apart (dR), so a step's scaling never overwrites what other threads read.
// (One wavefront on an 8 x 8 grid, with no barrier waits, measured twice as
// slow: each step's sixteen LDS updates per thread then run back to back.)
//   scaled = 1: x_j = sqrt(G_jj) is column j's norm after projection; it is
//     dependent if x_j < 1e-10 * norm0_j (or not finite/positive).  The
//     remaining columns are scaled to unit norm (Gt = S G S, S = diag(1/x)) and
//     factored, Gt = Rt^T Rt; a pivot below 1e-13 marks a column numerically
//     dependent on the ones before it.  Rinv = S Rt^{-1}, so X Rinv has
//     orthonormal columns.
//   scaled = 0: plain G = R^T R, Rinv = R^{-1}; a non-positive pivot sets dep[kb].
// dep[j] (j < kb) = 1 for dependent columns, dep[kb] = 1 if any, dep[kb+1] = 1 if
// ||R^{-1}||_2 <= 100 is not certain for the (scaled) factor (its smallest
// diagonal entry is below 0.01, or ||R^{-1}||_F exceeds 100): R^{-1} may then
// amplify the block's residual components along the basis by more than 100.
// R^{-1} comes from Gauss-Jordan elimination on [R | I] from the last row up.
constexpr int kCholP = 16;  // thread grid edge: kCholP^2 threads

// TT x TT entries per thread: kb <= 16 TT (TT = 2 up to kb = 32, so the
// per-step loops carry no tiles that are wholly out of range).
template <int TT>
__global__ void __launch_bounds__(kCholP * kCholP) k_chol_rinv(const double *__restrict__ G, int kb,
                                                   const double *__restrict__ norm0,
                                                   double *__restrict__ Rinv, int *__restrict__ dep,
                                                   int scaled) {
    constexpr int P = kCholP, NT = P * P, KM = P * TT;
    // R in the upper triangle of A; B = R^{-1} (upper) kept transposed in the
    // strict lower triangle of A, its diagonal in bd
    __shared__ double A[KM][KM + 1];
    __shared__ double bd[KM], dR[KM];  // diagonals of R^{-1} and of R
    __shared__ double s[KM];
    __shared__ int d[KM + 2];
    const int tid = threadIdx.x, ti = tid / P, tj = tid % P;
    if (tid < kb) {
        d[tid] = 0;
        bd[tid] = 1.0;
        if (scaled) {
            const double x = sqrt(G[tid * kb + tid]);
            const bool bad = !(x > 0.0) || !isfinite(x) || !(x >= 1e-10 * norm0[tid]);
            s[tid] = bad ? 0.0 : 1.0 / x;
            d[tid] = bad;
        } else {
            s[tid] = 1.0;
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < TT; ++a)
#pragma unroll
        for (int b = 0; b < TT; ++b) {
            const int i = ti + P * a, j = tj + P * b;
            if (i < kb && j < kb && j >= i) {
                double v = G[i * kb + j] * s[i] * s[j];
                if (scaled && (d[i] || d[j])) v = (i == j) ? 1.0 : 0.0;  // placeholder, result discarded
                A[i][j] = v;
            }
        }
    __syncthreads();
    // right-looking Cholesky, upper factor
    const double thr = scaled ? 1e-13 : 0.0;
    for (int k = 0; k < kb; ++k) {
        double pv = A[k][k];
        const bool badp = !(pv > thr) || !isfinite(pv);
        if (badp) pv = 1.0;
        const double piv = sqrt(pv);
        // R_kk goes to dR, so A[k][k] is not written while others read it
        if (tid == 0) {
            if (badp) d[k] = 1;
            dR[k] = piv;
        }
        if (tid > k && tid < kb) A[k][tid] /= piv;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < TT; ++a)
#pragma unroll
            for (int b = 0; b < TT; ++b) {
                const int i = ti + P * a, j = tj + P * b;
                if (i > k && j >= i && j < kb) A[i][j] -= A[k][i] * A[k][j];
            }
        __syncthreads();
    }
    // B = I below the diagonal: zero the strict lower triangle
#pragma unroll
    for (int a = 0; a < TT; ++a)
#pragma unroll
        for (int b = 0; b < TT; ++b) {
            const int i = ti + P * a, j = tj + P * b;
            if (j < i && i < kb) A[i][j] = 0.0;
        }
    __syncthreads();
    // Gauss-Jordan on [R | B] from the last row up: B(k, :) /= R_kk, then
    // B(i, :) -= R_ik B(k, :) for i < k; B ends as R^{-1}
    for (int k = kb - 1; k >= 0; --k) {
        const double rk = 1.0 / dR[k];
        if (tid == k) bd[k] *= rk;
        if (tid > k && tid < kb) A[tid][k] *= rk;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < TT; ++a)
#pragma unroll
            for (int b = 0; b < TT; ++b) {
                const int i = ti + P * a, j = tj + P * b;
                if (i < k && j >= k && j < kb) A[j][i] -= A[i][k] * (j == k ? bd[k] : A[j][k]);
            }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TT; ++a)
#pragma unroll
        for (int b = 0; b < TT; ++b) {
            const int i = ti + P * a, j = tj + P * b;
            if (i < kb && j < kb) Rinv[i * kb + j] = s[i] * (i < j ? A[j][i] : i == j ? bd[i] : 0.0);
        }
    // ||R^{-1}||_F^2 of the column-scaled factor, an upper bound of ||R^{-1}||_2^2:
    // per-thread sums over a fixed set of entries, then a fixed-order tree
    // (deterministic)
    __shared__ double fro[NT];
    {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < TT; ++a)
#pragma unroll
            for (int b = 0; b < TT; ++b) {
                const int i = ti + P * a, j = tj + P * b;
                if (i < kb && j < kb && i <= j) {
                    const double v = i < j ? A[j][i] : bd[i];
                    acc += v * v;
                }
            }
        fro[tid] = acc;
    }
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (tid < h) fro[tid] += fro[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        int any = 0;
        double rmin = 1.0;
        for (int j = 0; j < kb; ++j) {
            any |= d[j];
            if (!d[j]) rmin = fmin(rmin, dR[j]);
        }
        dep[kb] = any;
        // a second full pass unless ||R^{-1}||_2 <= 100 is certain: then V^T X
        // grew by at most 100 in the first pass, and since the scaled factor has
        // unit columns (||R||_2 <= sqrt(kb) <= 8) kappa(R) <= 800, so X^T X is
        // within about kappa^2 eps of I and one Newton-Schulz step suffices
        dep[kb + 1] = rmin < 0.01 || !(fro[0] <= 1e4);
    }
    if (tid < kb) dep[tid] = d[tid];
}

__global__ void k_h_insert(double *__restrict__ H, int64_t ldh, const double *__restrict__ C, int k,
                           int kb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= k * kb) return;
    const int i = e / kb, j = e % kb;
    const int c = k - kb + j;
    if (i < k - kb) {
        H[(int64_t)i * ldh + c] = C[e];
        H[(int64_t)c * ldh + i] = C[e];
    } else {
        const int a = i - (k - kb);
        H[(int64_t)i * ldh + c] = 0.5 * (C[e] + C[(int64_t)(k - kb + j) * kb + a]);
    }
}

__global__ void k_h_set_diag(double *__restrict__ H, int64_t ldh, const double *__restrict__ dg, int k) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int i = (int)(e / k), j = (int)(e % k);
    H[(int64_t)i * ldh + j] = (i == j) ? dg[i] : 0.0;
}

// C (m x n, ldc) = op(A) B with op(A) = A (m x k, lda) or A^T (A is k x m, lda)
// and B (k x n, ldb): 32 x 32 output tiles, 32-deep slices of both operands
// staged in LDS with coalesced loads; every output sums over k in ascending
// order.  Rows m .. m + mc - 1 of C are copied from S (lds) rows 0 .. mc - 1.
// For the small matrices of the deferred rotation (<= 512 on a side).
template <bool TA>
__global__ void __launch_bounds__(256) k_small_gemm(const double *__restrict__ A, int64_t lda,
                                                    const double *__restrict__ B, int64_t ldb,
                                                    double *__restrict__ C, int64_t ldc, int m, int n, int k,
                                                    const double *__restrict__ S, int64_t lds, int mc) {
    __shared__ double As[32][33], Bs[32][33];  // As[i][kk] = op(A)(i0 + i, k0 + kk)
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int kend = i0 < m ? k : 0;  // blocks wholly in the copied rows skip the product
    for (int k0 = 0; k0 < kend; k0 += 32) {
        for (int r = ty; r < 32; r += 8) {
            if (TA) {  // A row k0 + r, columns i0 + tx
                const int kk = k0 + r, i = i0 + tx;
                As[tx][r] = (kk < k && i < m) ? A[(int64_t)kk * lda + i] : 0.0;
            } else {   // A row i0 + r, columns k0 + tx
                const int i = i0 + r, kk = k0 + tx;
                As[r][tx] = (i < m && kk < k) ? A[(int64_t)i * lda + kk] : 0.0;
            }
            const int kk = k0 + r, j = j0 + tx;
            Bs[r][tx] = (kk < k && j < n) ? B[(int64_t)kk * ldb + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const double b = Bs[kk][tx];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += As[ty + 8 * q][kk] * b;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + ty + 8 * q, j = j0 + tx;
        if (j >= n) continue;
        if (i < m)
            C[(int64_t)i * ldc + j] = acc[q];
        else if (i < m + mc)
            C[(int64_t)i * ldc + j] = S[(int64_t)(i - m) * lds + j];
    }
}

}  // namespace

chebdav_status chol_rinv(const double *G, int kb, const double *norm0, double *Rinv, int *dep,
                         int scaled, hipStream_t st) {
    if (kb < 1 || kb > kMaxKb) return fail(CHEBDAV_EUNSUPPORTED, "block size %d outside [1, %d]", kb, kMaxKb);
    if (kb <= 2 * kCholP)
        hipLaunchKernelGGL(k_chol_rinv<2>, dim3(1), dim3(kCholP * kCholP), 0, st, G, kb, norm0, Rinv, dep, scaled);
    else
        hipLaunchKernelGGL(k_chol_rinv<kMaxKb / kCholP>, dim3(1), dim3(kCholP * kCholP), 0, st, G, kb, norm0, Rinv,
                           dep, scaled);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

chebdav_status h_insert(double *H, int64_t ldh, const double *C, int k, int kb, hipStream_t st) {
    const int total = k * kb;
    hipLaunchKernelGGL(k_h_insert, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, H, ldh, C, k, kb);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

chebdav_status h_set_diag(double *H, int64_t ldh, const double *d, int k, hipStream_t st) {
    if (k == 0) return CHEBDAV_OK;
    const int64_t total = (int64_t)k * k;
    hipLaunchKernelGGL(k_h_set_diag, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, H, ldh, d, k);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

// Deferred rotation of the search basis: the active block is kept as B Q, with
// B (n x kr, orthonormal, in HBM) and a small kr x ka matrix Q.
// New columns of H = [B Q, X]^T (A X) from Cf = [B, X]^T (A X):
// C(0:ka, :) = Q(:, 0:ka)^T Cf(0:kr, :), C(ka + t, :) = Cf(kr + t, :) (t < kb); C is
// (ka + kb) x kb contiguous.
chebdav_status proj_cols(const double *Q, int64_t ldq, const double *Cf, int kr, int ka, int kb, double *C,
                         hipStream_t st) {
    if (kb == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL(k_small_gemm<true>, dim3((unsigned)ceil_div(kb, 32), (unsigned)ceil_div(ka + kb, 32)), dim3(256),
                       0, st, Q, ldq, Cf, (int64_t)kb, C, (int64_t)kb, ka, kb, kr, Cf + (int64_t)kr * kb, (int64_t)kb,
                       kb);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

// Qn = [[Q, 0], [0, I_kb]] Y(:, 0:nc): Qn(0:kr, :) = Q(0:kr, 0:ka) Y(0:ka, 0:nc),
// Qn(kr + t, :) = Y(ka + t, 0:nc) (t < kb).
chebdav_status extend_basis(const double *Q, int64_t ldq, const double *Y, int64_t ldy, int kr, int ka, int kb,
                            int nc, double *Qn, int64_t ldn, hipStream_t st) {
    if (nc == 0 || kr + kb == 0) return CHEBDAV_OK;
    hipLaunchKernelGGL(k_small_gemm<false>, dim3((unsigned)ceil_div(nc, 32), (unsigned)ceil_div(kr + kb, 32)),
                       dim3(256), 0, st, Q, ldq, Y, ldy, Qn, ldn, kr, nc, ka, Y + (int64_t)ka * ldy, ldy, kb);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
