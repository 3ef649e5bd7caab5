// Tall-skinny QR by a tree of Householder factorizations (Sec. 3.3, distributed
// orthonormalization: the TSQR of Demmel et al. as its parallel-TSQR algorithm
// states it, with the row blocks of one GPU in place of processes).
//
// X (n x kb) is cut into row chunks of RC rows (KP the power of two >= kb, at
// least 8: 256 rows for KP = 64 and 32, 512 for 16, 1024 for 8), one workgroup
// each.  Every chunk is factored by Householder reflections (leaf level); its kb x kb R
// factors are stacked in chunk order into a (chunks * kb) x kb matrix, which is
// factored the same way (fan-in RC / kb >= 4), and so on until one chunk is
// left.  Its R is the R of X.  Q is formed top-down: the top chunk applies its
// reflectors to [I; 0], every lower chunk applies its own to [C; 0], where C is
// its kb-row block of the level above's Q.  The signs are fixed at the top so
// that R has a non-negative diagonal (then Q and R are the unique thin QR of a
// full-rank X).
//
// One chunk in one workgroup of NT threads (512 for KP = 64, else 256): thread
// (g, c) holds column c of the 32 consecutive rows g * 32 .. g * 32 + 31 of the
// chunk in registers.  For reflector j, column j reaches the other columns of a row group by a shuffle
// within the group's lanes, each thread forms the partial products of column j
// with its own column, and one barrier combines the row groups' partials through
// LDS in a fixed order.  The reflector is found from those sums alone:
//   alpha = x_jj, ||x_j||^2 = d_j, beta = -sign(alpha) ||x_j||,
//   v = (x_j - beta e_j) / (alpha - beta), tau = (beta - alpha) / beta,
//   v^T x_c = (d_c - beta x_jc) / (alpha - beta),
// where d_c is the product of the rows >= j of columns j and c.  A column that
// is zero from row j down gets tau = 0 (no reflection) and R_jj = 0.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kRpt = 32;  // rows of a chunk per thread
constexpr int kTsqrMaxKb = 64;
constexpr int kMaxLevels = 32;

__host__ __device__ constexpr int tsqr_threads(int kp) { return kp == 64 ? 512 : 256; }
__host__ __device__ constexpr int chunk_rows(int kp) { return tsqr_threads(kp) / kp * kRpt; }

// Householder factorization of chunk blockIdx.x of the m x kb matrix A
// (row-major, lda).  Writes the reflectors (strictly below the diagonal; the
// rows above hold R) to V (ldv; V may be A with the same ld: every chunk reads
// its rows before it writes them), tau to tau[chunk * kb + j], and the chunk's
// kb x kb R (zeros below the diagonal) to Rout + chunk * kb * kb.
template <int KP>
__global__ void __launch_bounds__(tsqr_threads(KP)) k_tsqr_factor(const double *A, int64_t lda, int64_t m, int kb,
                                                              double *V, int64_t ldv, double *__restrict__ tau,
                                                              double *__restrict__ Rout) {
    constexpr int G = tsqr_threads(KP) / KP, RC = G * kRpt;
    __shared__ double dpart[2][G][KP];
    __shared__ double rowj[2][KP];
    __shared__ double stau[KP];
    const int tid = threadIdx.x, g = tid / KP, c = tid % KP;
    const int ib = g * kRpt;  // first chunk row of this thread
    const int64_t chunk = blockIdx.x;
    const int64_t row0 = chunk * RC + ib;
    const bool colok = c < kb;
    // rows of this thread inside the matrix (0 for a column beyond kb)
    const int nr = colok ? (int)std::max<int64_t>(0, std::min<int64_t>(kRpt, m - row0)) : 0;
    double x[kRpt];
    {
        const double *p = A + (nr > 0 ? row0 * lda + c : 0);
#pragma unroll
        for (int t = 0; t < kRpt; ++t) x[t] = t < nr ? p[t * lda] : 0.0;
    }
    for (int j = 0; j < kb; ++j) {
        const int buf = j & 1;
        const int jt = j - ib;  // row j's slot in this thread's rows (if 0 <= jt < kRpt)
        double cj[kRpt];
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < kRpt; ++t) {
            const double v = __shfl(x[t], j, KP);
            cj[t] = (t >= jt) ? v : 0.0;
            d += cj[t] * x[t];
        }
        dpart[buf][g][c] = d;
        if (jt >= 0 && jt < kRpt) {
            double rj = x[0];
#pragma unroll
            for (int t = 1; t < kRpt; ++t) rj = (t == jt) ? x[t] : rj;
            rowj[buf][c] = rj;
        }
        __syncthreads();
        double nrm2 = 0.0, dc = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            nrm2 += dpart[buf][q][j];
            dc += dpart[buf][q][c];
        }
        const double alpha = rowj[buf][j];
        double beta = 0.0, tj = 0.0, scal = 0.0;
        if (nrm2 > 0.0) {
            const double nrm = sqrt(nrm2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tj = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        const double w = (dc - beta * rowj[buf][c]) * scal;  // v^T x_c
        const double tw = c > j ? tj * w : 0.0;
        const bool own = c == j;  // column j itself becomes (R_jj, v)
#pragma unroll
        for (int t = 0; t < kRpt; ++t) {
            const double vt = (t == jt) ? 1.0 : cj[t] * scal;
            const double upd = x[t] - tw * vt;
            const double mine = (t == jt) ? beta : (t > jt ? vt : x[t]);
            x[t] = own ? mine : upd;
        }
        if (tid == 0) stau[j] = tj;  // global stores wait until the end: none inside the loop
    }
    const int64_t m_here = m - chunk * RC;
    __syncthreads();
    if (tid < kb) tau[chunk * kb + tid] = stau[tid];
    {
        double *p = V + (nr > 0 ? row0 * ldv + c : 0);
#pragma unroll
        for (int t = 0; t < kRpt; ++t)
            if (t < nr) p[t * ldv] = x[t];
    }
    if (ib < kb && colok) {
        double *R = Rout + chunk * kb * kb;
#pragma unroll
        for (int t = 0; t < kRpt; ++t) {
            const int i = ib + t;
            if (i < kb) R[i * kb + c] = (c >= i && i < m_here) ? x[t] : 0.0;
        }
    }
}

// Q of chunk blockIdx.x: Y = H_0 H_1 ... H_{kb-1} [C; 0] with the chunk's
// reflectors (V, tau as written by k_tsqr_factor over the same m, kb), C the
// chunk's kb x kb block of the level above's Q (rows chunk * kb .. + kb - 1 of
// Cabove, ld kb), or the identity when Cabove is null (top level).  With sgn
// non-null (top level), column c is multiplied by the sign of sgn[c * kb + c]
// (the diagonal of the top R; +1 for zero).  Writes the chunk's m rows of Y
// (ldy; Y may be V with the same ld).
template <int KP>
__global__ void __launch_bounds__(tsqr_threads(KP)) k_tsqr_q(const double *V, int64_t ldv, const double *__restrict__ tau,
                                                         int64_t m, int kb, const double *__restrict__ Cabove,
                                                         const double *__restrict__ sgn, double *Y, int64_t ldy) {
    constexpr int G = tsqr_threads(KP) / KP, RC = G * kRpt;
    __shared__ double dpart[2][G][KP];
    __shared__ double stau[KP];
    const int tid = threadIdx.x, g = tid / KP, c = tid % KP;
    const int ib = g * kRpt;
    const int64_t chunk = blockIdx.x;
    if (tid < kb) stau[tid] = tau[chunk * kb + tid];
    const int64_t row0 = chunk * RC + ib;
    const bool colok = c < kb;
    const int nr = colok ? (int)std::max<int64_t>(0, std::min<int64_t>(kRpt, m - row0)) : 0;
    double x[kRpt], y[kRpt];
    {
        const double *p = V + (nr > 0 ? row0 * ldv + c : 0);
#pragma unroll
        for (int t = 0; t < kRpt; ++t) x[t] = t < nr ? p[t * ldv] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kRpt; ++t) {
        const int i = ib + t;
        double yt = 0.0;
        if (i < kb && t < nr) yt = Cabove ? Cabove[(chunk * kb + i) * kb + c] : (i == c ? 1.0 : 0.0);
        y[t] = yt;
    }
    for (int j = kb - 1; j >= 0; --j) {
        const int buf = j & 1;
        const int jt = j - ib;
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < kRpt; ++t) {
            const double v = __shfl(x[t], j, KP);
            const double vt = (t > jt) ? v : (t == jt ? 1.0 : 0.0);
            d += vt * y[t];
        }
        dpart[buf][g][c] = d;
        __syncthreads();
        double wc = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q) wc += dpart[buf][q][c];
        const double tw = stau[j] * wc;
#pragma unroll
        for (int t = 0; t < kRpt; ++t) {
            const double v = __shfl(x[t], j, KP);
            const double vt = (t > jt) ? v : (t == jt ? 1.0 : 0.0);
            y[t] -= tw * vt;
        }
    }
    double s = 1.0;
    if (sgn && colok && sgn[c * kb + c] < 0.0) s = -1.0;
    {
        double *p = Y + (nr > 0 ? row0 * ldy + c : 0);
#pragma unroll
        for (int t = 0; t < kRpt; ++t)
            if (t < nr) p[t * ldy] = s * y[t];
    }
}

// R (ldr) = diag(s) Rtop with s_i the sign of Rtop_ii (+1 for zero); zeros
// below the diagonal.
__global__ void k_tsqr_rsign(const double *__restrict__ Rtop, int kb, double *__restrict__ R, int64_t ldr) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kb * kb) return;
    const int i = e / kb, j = e % kb;
    const double s = Rtop[i * kb + i] < 0.0 ? -1.0 : 1.0;
    R[i * ldr + j] = j >= i ? s * Rtop[i * kb + j] : 0.0;
}

// Dependence flags from the R of a projected block, with the conventions of
// the scaled Cholesky QR: x_j = ||R(:, j)|| is column j's norm after
// projection, dependent when x_j < 1e-10 norm0_j (or not finite/positive);
// r_j = R_jj / x_j is its pivot in the column-scaled factor, dependent when
// r_j^2 <= 1e-13.  dep[kb] = any, dep[kb + 1] = smallest r_j of the others < 0.01.
__global__ void k_tsqr_dep(const double *__restrict__ R, int64_t ldr, int kb, const double *__restrict__ norm0,
                           int *__restrict__ dep) {
    __shared__ double piv[kTsqrMaxKb], cn[kTsqrMaxKb], fro[kTsqrMaxKb];
    __shared__ double xs[kTsqrMaxKb][kTsqrMaxKb + 1];  // column j of the inverse of R S^{-1} in xs[.][j]
    __shared__ int d[kTsqrMaxKb];
    const int j = threadIdx.x;
    if (j < kb) {
        double s = 0.0;
        for (int i = 0; i <= j; ++i) s += R[i * ldr + j] * R[i * ldr + j];
        const double x = sqrt(s);
        bool bad = !(x > 0.0) || !isfinite(x) || !(x >= 1e-10 * norm0[j]);
        const double r = bad ? 0.0 : R[j * ldr + j] / x;
        if (!bad && !(r * r > 1e-13)) bad = true;
        piv[j] = r;
        cn[j] = bad ? 1.0 : x;
        d[j] = bad;
        dep[j] = bad;
    }
    __syncthreads();
    // ||(R S^{-1})^{-1}||_F^2 with S = diag of R's column norms (an upper bound
    // of the squared 2-norm of the scaled factor's inverse): thread j solves for
    // column j by back-substitution
    if (j < kb) {
        double f = 0.0;
        const double rjj = piv[j];
        xs[j][j] = rjj != 0.0 ? 1.0 / rjj : 0.0;
        f = xs[j][j] * xs[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double acc = 0.0;
            for (int l = i + 1; l <= j; ++l) acc += (R[i * ldr + l] / cn[l]) * xs[l][j];
            const double rii = piv[i];
            xs[i][j] = rii != 0.0 ? -acc / rii : 0.0;
            f += xs[i][j] * xs[i][j];
        }
        fro[j] = f;
    }
    __syncthreads();
    if (j == 0) {
        int any = 0;
        double rmin = 1.0, f = 0.0;
        for (int i = 0; i < kb; ++i) {
            any |= d[i];
            if (!d[i]) rmin = fmin(rmin, piv[i]);
            f += fro[i];
        }
        dep[kb] = any;
        // a second pass (projection, then TSQR again) unless the inverse of the
        // scaled factor is certain to amplify components along V by at most 100
        dep[kb + 1] = rmin < 0.01 || !(f <= 1e4);
    }
}

int tsqr_kp(int kb) { return kb <= 8 ? 8 : kb <= 16 ? 16 : kb <= 32 ? 32 : 64; }

struct TsqrPlan {
    int levels = 0;               // number of levels (1 = the leaf is the top)
    int64_t m[kMaxLevels] = {};   // rows of the level's matrix
    int64_t p[kMaxLevels] = {};   // chunks of the level
};

TsqrPlan tsqr_plan(int64_t n, int kb) {
    TsqrPlan pl;
    const int rc = chunk_rows(tsqr_kp(kb));
    int64_t m = n;
    for (;;) {
        pl.m[pl.levels] = m;
        pl.p[pl.levels] = ceil_div(m, rc);
        const int64_t p = pl.p[pl.levels];
        ++pl.levels;
        if (p == 1) break;
        m = p * kb;
    }
    return pl;
}

struct TsqrWs {
    double *stack[kMaxLevels] = {};  // level l >= 1: its m x kb input, then reflectors, then Q
    double *tau[kMaxLevels] = {};
    double *rtop = nullptr;
};

TsqrWs tsqr_layout(Arena &a, const TsqrPlan &pl, int kb) {
    TsqrWs s;
    for (int l = 1; l < pl.levels; ++l) s.stack[l] = a.take<double>((size_t)pl.m[l] * kb);
    for (int l = 0; l < pl.levels; ++l) s.tau[l] = a.take<double>((size_t)pl.p[l] * kb);
    s.rtop = a.take<double>((size_t)kb * kb);
    return s;
}

template <int KP>
void launch_factor(const TsqrPlan &pl, const TsqrWs &s, int l, const double *A, int64_t lda, double *V,
                   int64_t ldv, int kb, hipStream_t st) {
    double *rout = (l + 1 < pl.levels) ? s.stack[l + 1] : s.rtop;
    hipLaunchKernelGGL(k_tsqr_factor<KP>, dim3((unsigned)pl.p[l]), dim3(tsqr_threads(KP)), 0, st, A, lda, pl.m[l], kb, V,
                       ldv, s.tau[l], rout);
}

template <int KP>
void launch_q(const TsqrPlan &pl, const TsqrWs &s, int l, const double *V, int64_t ldv, double *Y, int64_t ldy,
              int kb, hipStream_t st) {
    const bool top = l + 1 == pl.levels;
    hipLaunchKernelGGL(k_tsqr_q<KP>, dim3((unsigned)pl.p[l]), dim3(tsqr_threads(KP)), 0, st, V, ldv, s.tau[l], pl.m[l], kb,
                       top ? nullptr : s.stack[l + 1], top ? s.rtop : nullptr, Y, ldy);
}

chebdav_status check_shape(int64_t n, int kb) {
    if (kb < 1 || kb > kTsqrMaxKb) return fail(CHEBDAV_EUNSUPPORTED, "TSQR block width %d outside [1, %d]", kb, kTsqrMaxKb);
    if (n < kb) return fail(CHEBDAV_EINVAL, "TSQR needs n >= kb (n = %lld, kb = %d)", (long long)n, kb);
    if (tsqr_plan(n, kb).levels >= kMaxLevels) return fail(CHEBDAV_EUNSUPPORTED, "TSQR tree too deep");
    return CHEBDAV_OK;
}

}  // namespace

chebdav_status tsqr_ws_bytes(int64_t n, int kb, size_t *bytes) {
    CD_TRY(check_shape(n, kb));
    Arena a;
    a.counting = true;
    (void)tsqr_layout(a, tsqr_plan(n, kb), kb);
    *bytes = a.used + 256;
    return CHEBDAV_OK;
}

chebdav_status tsqr_factor(const double *X, int64_t ldx, int64_t n, int kb, double *Vleaf, int64_t ldv, double *R,
                           int64_t ldr, void *ws, size_t ws_bytes, hipStream_t st) {
    size_t need = 0;
    CD_TRY(tsqr_ws_bytes(n, kb, &need));
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "TSQR workspace too small (%zu < %zu)", ws_bytes, need);
    if (ldx < kb || ldv < kb || ldr < kb) return fail(CHEBDAV_EINVAL, "TSQR leading dimension below kb");
    const TsqrPlan pl = tsqr_plan(n, kb);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const TsqrWs s = tsqr_layout(a, pl, kb);
    const int kp = tsqr_kp(kb);
    for (int l = 0; l < pl.levels; ++l) {
        const double *A = l == 0 ? X : s.stack[l];
        double *V = l == 0 ? Vleaf : s.stack[l];
        const int64_t lda = l == 0 ? ldx : kb, lv = l == 0 ? ldv : kb;
        switch (kp) {
            case 8: launch_factor<8>(pl, s, l, A, lda, V, lv, kb, st); break;
            case 16: launch_factor<16>(pl, s, l, A, lda, V, lv, kb, st); break;
            case 32: launch_factor<32>(pl, s, l, A, lda, V, lv, kb, st); break;
            default: launch_factor<64>(pl, s, l, A, lda, V, lv, kb, st); break;
        }
        CD_LAUNCH_CHECK();
    }
    if (R) {
        hipLaunchKernelGGL(k_tsqr_rsign, dim3((unsigned)ceil_div((int64_t)kb * kb, 256)), dim3(256), 0, st, s.rtop, kb, R,
                           ldr);
        CD_LAUNCH_CHECK();
    }
    return CHEBDAV_OK;
}

chebdav_status tsqr_form_q(int64_t n, int kb, const double *Vleaf, int64_t ldv, double *Q, int64_t ldq, void *ws,
                           size_t ws_bytes, hipStream_t st) {
    size_t need = 0;
    CD_TRY(tsqr_ws_bytes(n, kb, &need));
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "TSQR workspace too small (%zu < %zu)", ws_bytes, need);
    if (ldv < kb || ldq < kb) return fail(CHEBDAV_EINVAL, "TSQR leading dimension below kb");
    const TsqrPlan pl = tsqr_plan(n, kb);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const TsqrWs s = tsqr_layout(a, pl, kb);
    const int kp = tsqr_kp(kb);
    for (int l = pl.levels - 1; l >= 0; --l) {
        const double *V = l == 0 ? Vleaf : s.stack[l];
        double *Y = l == 0 ? Q : s.stack[l];
        const int64_t lv = l == 0 ? ldv : kb, ly = l == 0 ? ldq : kb;
        switch (kp) {
            case 8: launch_q<8>(pl, s, l, V, lv, Y, ly, kb, st); break;
            case 16: launch_q<16>(pl, s, l, V, lv, Y, ly, kb, st); break;
            case 32: launch_q<32>(pl, s, l, V, lv, Y, ly, kb, st); break;
            default: launch_q<64>(pl, s, l, V, lv, Y, ly, kb, st); break;
        }
        CD_LAUNCH_CHECK();
    }
    return CHEBDAV_OK;
}

chebdav_status tsqr_dep(const double *R, int64_t ldr, int kb, const double *norm0, int *dep, hipStream_t st) {
    if (kb < 1 || kb > kTsqrMaxKb) return fail(CHEBDAV_EUNSUPPORTED, "TSQR block width %d outside [1, %d]", kb, kTsqrMaxKb);
    hipLaunchKernelGGL(k_tsqr_dep, dim3(1), dim3(64), 0, st, R, ldr, kb, norm0, dep);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
