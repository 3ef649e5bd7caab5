// Symmetric eigendecomposition H = Y diag(w) Y^T of the small Rayleigh-quotient
// matrix (Alg. 2 step 9), ascending.  Pipeline:
//   1. Householder tridiagonalization Q^T H Q = T (one workgroup; the working
//      matrix in registers up to n = 160, else in L2);
//   2. eigenvalues of T by multisection on Sturm counts, one wavefront per
//      eigenvalue (64 points per round);
//   3. eigenvectors of T by inverse iteration with the LU factorization (with
//      partial pivoting) of T - w I, one wavefront per eigenvector, factors in LDS;
//   4. modified Gram-Schmidt inside tight clusters (gap <= 1e-6 ||T||);
//   5. back-transformation Y = Q Z, one wavefront per eigenvector;
//   6. one Newton-Schulz step Y <- Y (3 I - Y^T Y)/2 restores orthogonality to
//      rounding level (inverse-iteration vectors of distinct eigenvalues are
//      orthogonal only to about eps ||T|| / gap).
#include <cfloat>

#include "device_util.h"
#include "internal.h"

namespace chebdav {
namespace {

constexpr int kMaxN = 1024;
constexpr int kRegMaxN = 160;  // working matrix in registers up to this size
constexpr double kEps = DBL_EPSILON * 0.5;
constexpr double kTightRel = 1e-6;

struct EigWs {
    double *A, *Vh, *Zv;
    double *d, *e, *tau, *w, *par, *G, *Bm, *T, *part;
};

EigWs eig_layout(Arena &a, int n) {
    EigWs s;
    const size_t nn = (size_t)n * n;
    s.A = a.take<double>(nn);
    s.Vh = a.take<double>(nn);
    s.Zv = a.take<double>(nn);
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

// Householder step k of the lower tridiagonalization, on the n x n working
// matrix A (row-major, leading dimension n): v = x - alpha e1 for the column
// x = A(k+1:n, k), p = tau A v, w = p - (tau/2)(p^T v) v, A <- A - v w^T - w v^T.
// The update is done by rows (each wavefront owns rows i = wave, wave + nw, ...;
// lanes run over columns), the product A v by columns (no cross-lane sums).
__device__ __forceinline__ void tridiag_run(double *A, const double *__restrict__ H, int64_t ldh, int n,
                                            double *__restrict__ Vh, double *__restrict__ d,
                                            double *__restrict__ e, double *__restrict__ tau,
                                            double *v, double *wsh, double *red) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = lane_id(), wv = tid / kWave, nw = nt / kWave;
    for (int i = wv; i < n; i += nw)
        for (int j = lane; j < n; j += kWave) A[i * n + j] = H[(int64_t)i * ldh + j];
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        const int base = (k + 1) * n + (k + 1);  // A(k+1, k+1)
        double part = 0.0;
        for (int i = tid; i < m; i += nt) {
            const double xi = A[(k + 1 + i) * n + k];
            v[i] = xi;
            if (i > 0) part += xi * xi;
        }
        const double ss = block_sum(part);  // also makes v visible
        const double x0 = v[0];
        const double dk = A[k * n + k];
        if (ss == 0.0) {
            if (tid == 0) {
                tau[k] = 0.0;
                e[k] = x0;
                d[k] = dk;
            }
            for (int i = tid; i < m; i += nt) Vh[k * n + i] = 0.0;
            __syncthreads();
            continue;
        }
        const double alpha = -copysign(sqrt(x0 * x0 + ss), x0);
        const double v0 = x0 - alpha;
        const double t = 2.0 / (v0 * v0 + ss);
        if (tid == 0) {
            tau[k] = t;
            e[k] = alpha;
            d[k] = dk;
        }
        // p = t A v (A symmetric, so p_i = t sum_j A(j, i) v_j): threads own
        // columns i, JG groups of threads split the j range, partial sums meet in red
        if (tid == 0) v[0] = v0;
        __syncthreads();
        {
            constexpr int JG = 4;
            const int cw = nt / JG;
            const int g = tid / cw, c = tid % cw;
            for (int i0 = 0; i0 < m; i0 += cw) {
                const int i = i0 + c;
                double sacc = 0.0;
                if (i < m)
                    for (int j = g; j < m; j += JG) sacc += A[base + j * n + i] * v[j];
                red[g * cw + c] = sacc;
                __syncthreads();
                if (g == 0 && i < m) wsh[i] = t * (red[c] + red[cw + c] + red[2 * cw + c] + red[3 * cw + c]);
                __syncthreads();
            }
        }
        part = 0.0;
        for (int i = tid; i < m; i += nt) part += wsh[i] * v[i];
        const double K = 0.5 * t * block_sum(part);
        for (int i = tid; i < m; i += nt) wsh[i] -= K * v[i];
        __syncthreads();
        for (int i = wv; i < m; i += nw) {
            double *row = A + base + i * n;
            const double vi = v[i], wi = wsh[i];
            for (int j = lane; j < m; j += kWave) row[j] -= vi * wsh[j] + wi * v[j];
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

// Working matrix in global memory (L2-resident), any n <= kMaxN.
__global__ void __launch_bounds__(512) k_tridiag(const double *__restrict__ H, int64_t ldh, int n,
                                                 double *Ag, double *__restrict__ Vh, double *__restrict__ d,
                                                 double *__restrict__ e, double *__restrict__ tau) {
    __shared__ double v[kMaxN], wsh[kMaxN], red[512];
    tridiag_run(Ag, H, ldh, n, Vh, d, e, tau, v, wsh, red);
}

// Sum over a group of P consecutive lanes (P = 16: DPP row rotations; P = 32:
// plus one exchange between the two 16-lane rows), the same value in every lane.
// The exchange is v_permlane16_swap on both halves of the double (a VALU op,
// no LDS round trip): called with the same value twice it returns, in every
// lane of a 32-lane half, the even row's sum as x and the odd row's as y, so
// x + y is the group sum, added in the same order in every lane.
template <int P>
__device__ inline double group_sum(double v) {
    v = row16_sum(v);
    if constexpr (P == 32) {
        const uint64_t u = (uint64_t)__double_as_longlong(v);
        const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
        const double x = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
        const double y = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
        v = x + y;
    }
    return v;
}

// Register-resident variant for n <= P T: the working matrix is spread over a
// P x P thread grid (P = 32: 1024 threads), thread (pc, pr) = (tid / P, tid % P)
// holding A(pr + P a, pc + P b) for a, b < T, so a group of P lanes (one pc) owns
// whole columns.  A step k then needs two barriers: the row group that owns
// column k forms the reflector from its registers (sums over its 16 lanes by
// DPP row rotations) and publishes v; every thread forms its column sums of
// A v (row rotations again; A is symmetric, so column sums are p), the row
// groups publish p and their share of p^T v; every thread then updates its
// entries of the columns after k.  Tiles whose rows or columns are all finished
// are skipped.  Nothing goes to global memory inside the loop (a store there
// makes the next step wait for it): reflector k stays in column k below the
// diagonal, which later steps no longer update, and d, e, tau stay in LDS until
// the end.
template <int P, int T>
__global__ void __launch_bounds__(P * P) k_tridiag_reg(const double *__restrict__ H, int64_t ldh, int n,
                                                       double *__restrict__ Vh, double *__restrict__ d,
                                                       double *__restrict__ e, double *__restrict__ tau) {
    constexpr int NV = P * T;
    __shared__ double vs[NV], ps[NV], kp[P], scal[2];
    __shared__ double sd[NV], se[NV], stau[NV];
    const int tid = threadIdx.x, pc = tid / P, pr = tid % P;
    double A[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const int i = pr + P * a, j = pc + P * b;
            A[a][b] = (i < n && j < n) ? H[(int64_t)i * ldh + j] : 0.0;
        }
    for (int k = 0; k + 2 < n; ++k) {
        if (pc == k % P) {
            // column k of the working matrix, rows pr + 16 a
            const int bk = k / P;
            double col[T];
#pragma unroll
            for (int a = 0; a < T; ++a) {
                double v = 0.0;
#pragma unroll
                for (int b = 0; b < T; ++b) v = (b == bk) ? A[a][b] : v;
                col[a] = v;
            }
            double part = 0.0, x0 = 0.0, dk = 0.0;
#pragma unroll
            for (int a = 0; a < T; ++a) {
                const int i = pr + P * a;
                if (i > k + 1 && i < n) part += col[a] * col[a];
                if (i == k + 1) x0 = col[a];
                if (i == k) dk = col[a];
            }
            const double ss = group_sum<P>(part);
            x0 = group_sum<P>(x0);  // one lane holds it, the others add zeros
            dk = group_sum<P>(dk);
            double t = 0.0, v0 = 0.0, alpha = x0;
            if (ss != 0.0) {
                alpha = -copysign(sqrt(x0 * x0 + ss), x0);
                v0 = x0 - alpha;
                t = 2.0 / (v0 * v0 + ss);
            }
#pragma unroll
            for (int a = 0; a < T; ++a) {
                const int i = pr + P * a;
                double v = 0.0;
                if (t != 0.0 && i > k && i < n) v = (i == k + 1) ? v0 : col[a];
                vs[i] = v;
                if (i == k + 1) {  // column k keeps the reflector: v0 here, x below
#pragma unroll
                    for (int b = 0; b < T; ++b)
                        if (b == bk) A[a][b] = v0;
                }
            }
            if (pr == 0) {
                scal[0] = t;
                stau[k] = t;
                se[k] = alpha;
                sd[k] = dk;
            }
        }
        __syncthreads();
        const double t = scal[0];
        if (t == 0.0) {  // uniform: the reflector is the identity
            __syncthreads();  // everyone has read scal before the next step rewrites it
            continue;
        }
        double vr[T], vc[T], q[T];
#pragma unroll
        for (int a = 0; a < T; ++a) vr[a] = vs[pr + P * a];
#pragma unroll
        for (int b = 0; b < T; ++b) vc[b] = vs[pc + P * b];
        // p_j = t sum_i A(i, j) v_i for this row group's columns j = pc + 16 b
        double kpart = 0.0;
#pragma unroll
        for (int b = 0; b < T; ++b) {
            q[b] = 0.0;
            if (P * (b + 1) - 1 <= k) continue;  // columns of this tile are all finished
            double sacc = 0.0;
#pragma unroll
            for (int a = 0; a < T; ++a)
                if (P * (a + 1) - 1 > k) sacc += A[a][b] * vr[a];
            const double gs = group_sum<P>(sacc);
            q[b] = (pc + P * b > k) ? t * gs : 0.0;  // finished columns hold reflectors
            kpart += q[b] * vc[b];
        }
#pragma unroll
        for (int b = 0; b < T; ++b)
            if (pr == b) ps[pc + P * b] = q[b];
        if (pr == 0) kp[pc] = kpart;
        __syncthreads();
        // w = p - (t/2)(p^T v) v;  A <- A - v w^T - w v^T
        // p^T v: the P row-group shares, summed across the P lanes of a group.
        // Finished columns j <= k need no guard: there q_j = 0 and v_j = 0, so
        // w_j = 0 and their entries (the stored reflectors) change by exactly 0;
        // finished rows likewise have v_i = 0 and w_i = 0.
        const double ktot = group_sum<P>(kp[pr]);
        const double K = 0.5 * t * ktot;
#pragma unroll
        for (int a = 0; a < T; ++a) {
            if (P * (a + 1) - 1 <= k) continue;
            const double wr = ps[pr + P * a] - K * vr[a];
#pragma unroll
            for (int b = 0; b < T; ++b)
                if (P * (b + 1) - 1 > k) A[a][b] -= vr[a] * (q[b] - K * vc[b]) + wr * vc[b];
        }
    }
    __syncthreads();
    // reflectors (zero for an identity step), d, e, tau of the n - 2 steps
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const int i = pr + P * a, j = pc + P * b;
            if (j + 2 < n && i > j && i < n) Vh[(int64_t)j * n + (i - j - 1)] = stau[j] != 0.0 ? A[a][b] : 0.0;
        }
    for (int k = tid; k + 2 < n; k += P * P) {
        d[k] = sd[k];
        e[k] = se[k];
        tau[k] = stau[k];
    }
    // trailing 2 x 2 block (or the 1 x 1 matrix)
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const int i = pr + P * a, j = pc + P * b;
            if (n >= 2) {
                if (i == n - 2 && j == n - 2) d[n - 2] = A[a][b];
                if (i == n - 1 && j == n - 2) e[n - 2] = A[a][b];
                if (i == n - 1 && j == n - 1) {
                    d[n - 1] = A[a][b];
                    e[n - 1] = 0.0;
                }
            } else if (i == 0 && j == 0) {
                d[0] = A[a][b];
                e[0] = 0.0;
            }
        }
}

// 1/q from the hardware reciprocal refined by one Newton step (relative error
// a few units in the last place: enough for a backward-stable Sturm count).
__device__ inline double recip(double q) {
    const double r = __builtin_amdgcn_rcp(q);
    return fma(r, fma(-q, r, 1.0), r);
}

// Number of eigenvalues of T smaller than x (Sturm sequence), from d and the
// squared off-diagonal e2 (e2[i] = e[i]^2) in LDS; eight entries are read ahead
// of the recurrence, whose latency then sets the pace.
__device__ inline int sturm(const double *d, const double *e2, int n, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    int i = 1;
    for (; i + 7 < n; i += 8) {
        double dv[8], ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dv[u] = d[i + u];
            ev[u] = e2[i + u - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            q = dv[u] - x - ev[u] * recip(q);
            if (fabs(q) < pivmin) q = -pivmin;
            c += q < 0.0;
        }
    }
    for (; i < n; ++i) {
        q = d[i] - x - e2[i - 1] * recip(q);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Multisection: one wavefront per eigenvalue j; each round the 64 lanes count
// eigenvalues below 64 interior points of [lo, hi] and the bracket shrinks to
// the first sub-interval whose right end has more than j eigenvalues below it.
__global__ void __launch_bounds__(256) k_bisect(const double *__restrict__ d, const double *__restrict__ e,
                                                int n, double *__restrict__ w, double *__restrict__ par) {
    __shared__ double sd[kMaxN], se2[kMaxN];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        sd[i] = d[i];
        se2[i] = i + 1 < n ? e[i] * e[i] : 0.0;
    }
    __syncthreads();
    const int lane = lane_id();
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= n) return;
    double gl = DBL_MAX, gu = -DBL_MAX, emax2 = 0.0;
    for (int i = lane; i < n; i += kWave) {
        const double el = i > 0 ? fabs(e[i - 1]) : 0.0;
        const double er = i + 1 < n ? fabs(e[i]) : 0.0;
        gl = fmin(gl, d[i] - el - er);
        gu = fmax(gu, d[i] + el + er);
        emax2 = fmax(emax2, er * er);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        gl = fmin(gl, __shfl_xor(gl, o, kWave));
        gu = fmax(gu, __shfl_xor(gu, o, kWave));
        emax2 = fmax(emax2, __shfl_xor(emax2, o, kWave));
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double atol = 2.0 * kEps * tnorm + pivmin;
    double lo = gl - atol - 2.0 * kEps * tnorm, hi = gu + atol + 2.0 * kEps * tnorm;
    for (int round = 0; round < 64; ++round) {
        if (hi - lo <= atol) break;
        const double x = lo + (hi - lo) * ((double)(lane + 1) / (double)(kWave + 1));
        const bool above = sturm(sd, se2, n, x, pivmin) > j;
        const uint64_t mask = __ballot(above);
        const double xprev = __shfl_up(x, 1, kWave);
        if (mask == 0ull) {
            const double xl = __shfl(x, kWave - 1, kWave);
            if (!(xl > lo)) break;
            lo = xl;
        } else {
            const int l = __ffsll((unsigned long long)mask) - 1;
            const double xh = __shfl(x, l, kWave);
            const double xlo = __shfl(xprev, l, kWave);
            const double nlo = l > 0 ? xlo : lo;
            if (!(xh < hi) && !(nlo > lo)) break;
            hi = xh;
            lo = nlo;
        }
    }
    if (lane == 0) {
        w[j] = 0.5 * (lo + hi);
        if (j == 0) {
            par[0] = tnorm;
            par[1] = pivmin;
        }
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

// Inverse iteration: one wavefront per eigenvector with the LU factors of
// T - lambda I in LDS; lane 0 runs the sequential factorization and solves, the
// wavefront shares the vector operations.
__global__ void __launch_bounds__(64) k_inviter(const double *__restrict__ d, const double *__restrict__ e,
                                                int n, const double *__restrict__ w,
                                                const double *__restrict__ par, double *__restrict__ Zv) {
    extern __shared__ double sm[];
    double *dl = sm, *dd = sm + n, *du = sm + 2 * n, *du2 = sm + 3 * n, *x = sm + 4 * n;
    int *ipiv = reinterpret_cast<int *>(sm + 6 * n);
    const int j = blockIdx.x;
    const int lane = lane_id();
    if (n == 1) {
        if (lane == 0) Zv[0] = 1.0;
        return;
    }
    const double tnorm = par[0];
    const double tight = kTightRel * tnorm;
    const double pert = 10.0 * kEps * fmax(tnorm, DBL_MIN);
    int pos = 0;
    for (int i = j - 1; i >= 0 && w[i + 1] - w[i] <= tight; --i) ++pos;
    const double lam = w[j] + pert * pos;
    const double tiny = kEps * fmax(tnorm, DBL_MIN);
    for (int i = lane; i < n; i += kWave) {
        dd[i] = d[i] - lam;
        dl[i] = i + 1 < n ? e[i] : 0.0;
        du[i] = i + 1 < n ? e[i] : 0.0;
        du2[i] = 0.0;
        x[i] = hash_unit((uint32_t)i, (uint32_t)j);
    }
    __syncthreads();
    double *rdd = sm + 5 * n;
    if (lane == 0) {
        // LU with partial pivoting of the tridiagonal T - lam I; the running
        // diagonal and superdiagonal entries are carried in registers.  The
        // loops below read eight entries ahead into registers (the arrays share
        // one LDS buffer, so the compiler cannot move reads above the writes).
        double ddi = dd[0], dui = du[0];
        auto lu_step = [&](int i, double b, double ddn, double dun) {
            if (fabs(ddi) >= fabs(b)) {
                ipiv[i] = i;
                const double piv = ddi != 0.0 ? ddi : tiny;
                dd[i] = piv;
                const double f = b * recip(piv);
                dl[i] = f;
                du[i] = dui;
                ddi = ddn - f * dui;
                dui = dun;
            } else {
                ipiv[i] = i + 1;
                const double f = ddi * recip(b);
                dd[i] = b;
                dl[i] = f;
                du[i] = ddn;
                ddi = dui - f * ddn;
                if (i + 2 < n) du2[i] = dun;
                dui = -f * dun;
            }
        };
        int i = 0;
        for (; i + 9 < n; i += 8) {
            double bl[8], dn[8], un[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                bl[u] = dl[i + u];
                dn[u] = dd[i + u + 1];
                un[u] = du[i + u + 1];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) lu_step(i + u, bl[u], dn[u], un[u]);
        }
        for (; i + 1 < n; ++i) lu_step(i, dl[i], dd[i + 1], i + 2 < n ? du[i + 1] : 0.0);
        dd[n - 1] = ddi != 0.0 ? ddi : tiny;
    }
    __syncthreads();
    for (int i = lane; i < n; i += kWave) rdd[i] = 1.0 / dd[i];
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
        if (lane == 0) {
            // forward elimination with the row interchanges (x[i] carried in a register)
            double xi = x[0];
            auto fwd_step = [&](int i, double f, double xn, int pv) {
                if (pv == i) {
                    x[i] = xi;
                    xi = xn - f * xi;
                } else {
                    x[i] = xn;
                    xi = xi - f * xn;
                }
            };
            int i = 0;
            for (; i + 8 < n; i += 8) {
                double fv[8], xv[8];
                int pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    fv[u] = dl[i + u];
                    xv[u] = x[i + u + 1];
                    pv[u] = ipiv[i + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) fwd_step(i + u, fv[u], xv[u], pv[u]);
            }
            for (; i + 1 < n; ++i) fwd_step(i, dl[i], x[i + 1], ipiv[i]);
            x[n - 1] = xi;
            // back substitution with U (diagonal dd, superdiagonals du, du2)
            double xb = x[n - 1] * rdd[n - 1];
            x[n - 1] = xb;
            double xa = (x[n - 2] - du[n - 2] * xb) * rdd[n - 2];
            x[n - 2] = xa;
            int r = n - 3;
            for (; r - 7 >= 0; r -= 8) {
                double xr[8], dv[8], d2[8], rv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    xr[u] = x[r - u];
                    dv[u] = du[r - u];
                    d2[u] = du2[r - u];
                    rv[u] = rdd[r - u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double xv = (xr[u] - dv[u] * xa - d2[u] * xb) * rv[u];
                    x[r - u] = xv;
                    xb = xa;
                    xa = xv;
                }
            }
            for (; r >= 0; --r) {
                const double xv = (x[r] - du[r] * xa - du2[r] * xb) * rdd[r];
                x[r] = xv;
                xb = xa;
                xa = xv;
            }
        }
        __syncthreads();
        double mx = 0.0;
        for (int i = lane; i < n; i += kWave) mx = fmax(mx, fabs(x[i]));
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
        const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
        double s2 = 0.0;
        for (int i = lane; i < n; i += kWave) {
            const double v = x[i] * sc;
            s2 += v * v;
        }
        s2 = wave_sum(s2);
        const double nr = sc / sqrt(s2);
        for (int i = lane; i < n; i += kWave) x[i] *= nr;
        __syncthreads();
    }
    for (int i = lane; i < n; i += kWave) Zv[(int64_t)j * n + i] = x[i];
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
// The reflectors are loaded D steps ahead of their use (a ring of D register
// blocks) and tau sits in registers, read out lane by lane, so that a step
// waits on neither memory nor the scalar cache.
template <int kTpl>
__global__ void __launch_bounds__(256) k_backtransform(const double *__restrict__ Vh,
                                                       const double *__restrict__ tau,
                                                       const double *__restrict__ Zv, int n,
                                                       double *__restrict__ Y, int64_t ldy) {
    constexpr int D = kTpl <= 2 ? 8 : kTpl <= 4 ? 4 : 2;
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= n) return;
    const int lane = lane_id();
    double z[kTpl], tl[kTpl];
#pragma unroll
    for (int t = 0; t < kTpl; ++t) {
        const int i = lane + t * kWave;
        z[t] = i < n ? Zv[(int64_t)j * n + i] : 0.0;
        tl[t] = i + 2 < n ? tau[i] : 0.0;
    }
    auto load_v = [&](int k, double (&dst)[kTpl]) {
        const double *vk = Vh + (int64_t)k * n - (k + 1);  // vk[i] for i in [k+1, n)
#pragma unroll
        for (int t = 0; t < kTpl; ++t) {
            const int i = lane + t * kWave;
            dst[t] = (i > k && i < n) ? vk[i] : 0.0;
        }
    };
    double vb[D][kTpl];
#pragma unroll
    for (int u = 0; u < D; ++u)
        if (n - 3 - u >= 0) load_v(n - 3 - u, vb[u]);
    for (int k = n - 3; k >= 0; k -= D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int kk = k - u;
            if (kk < 0) break;
            double tv = tl[0];
#pragma unroll
            for (int t = 1; t < kTpl; ++t) tv = (t == (kk >> 6)) ? tl[t] : tv;
            const double tk = read_lane(tv, kk & (kWave - 1));
            if (tk != 0.0) {
                double dot = 0.0;
#pragma unroll
                for (int t = 0; t < kTpl; ++t) dot += vb[u][t] * z[t];
                const double sfac = tk * wave_sum(dot);
#pragma unroll
                for (int t = 0; t < kTpl; ++t) z[t] -= sfac * vb[u][t];
            }
            if (kk - D >= 0) load_v(kk - D, vb[u]);
        }
    }
#pragma unroll
    for (int t = 0; t < kTpl; ++t) {
        const int i = lane + t * kWave;
        if (i < n) Y[(int64_t)i * ldy + j] = z[t];
    }
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
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "eig workspace too small (%zu < %zu)", ws_bytes, need);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    EigWs s = eig_layout(a, n);
    if (n <= kRegMaxN) {
        // 16 x 16 grid up to n = 64 and above 128 (a 32 x 32 grid would spill
        // there), 32 x 32 grid for 64 < n <= 128 (measured faster)
        const dim3 b256(256), b1024(1024);
        if (n <= 32)
            hipLaunchKernelGGL((k_tridiag_reg<16, 2>), dim3(1), b256, 0, st, H, ldh, n, s.Vh, s.d, s.e, s.tau);
        else if (n <= 64)
            hipLaunchKernelGGL((k_tridiag_reg<16, 4>), dim3(1), b256, 0, st, H, ldh, n, s.Vh, s.d, s.e, s.tau);
        else if (n <= 96)
            hipLaunchKernelGGL((k_tridiag_reg<32, 3>), dim3(1), b1024, 0, st, H, ldh, n, s.Vh, s.d, s.e, s.tau);
        else if (n <= 128)
            hipLaunchKernelGGL((k_tridiag_reg<32, 4>), dim3(1), b1024, 0, st, H, ldh, n, s.Vh, s.d, s.e, s.tau);
        else
            hipLaunchKernelGGL((k_tridiag_reg<16, 10>), dim3(1), b256, 0, st, H, ldh, n, s.Vh, s.d, s.e, s.tau);
    } else
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(512), 0, st, H, ldh, n, s.A, s.Vh, s.d, s.e, s.tau);
    CD_LAUNCH_CHECK();
    const unsigned g64 = (unsigned)ceil_div(n, 64);
    hipLaunchKernelGGL(k_bisect, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, s.d, s.e, n, s.w, s.par);
    CD_LAUNCH_CHECK();
    const size_t inv_lds = sizeof(double) * 6 * n + sizeof(int) * n;
    hipLaunchKernelGGL(k_inviter, dim3(n), dim3(64), inv_lds, st, s.d, s.e, n, s.w, s.par, s.Zv);
    CD_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cluster_mgs, dim3(n), dim3(256), 0, st, s.w, s.par, n, s.Zv);
    CD_LAUNCH_CHECK();
    {
        const dim3 gb((unsigned)ceil_div(n, 4));
        switch ((int)ceil_div(n, kWave)) {
            case 1: hipLaunchKernelGGL(k_backtransform<1>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 2: hipLaunchKernelGGL(k_backtransform<2>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 3: hipLaunchKernelGGL(k_backtransform<3>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 4: hipLaunchKernelGGL(k_backtransform<4>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 5: hipLaunchKernelGGL(k_backtransform<5>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 6: hipLaunchKernelGGL(k_backtransform<6>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 7: hipLaunchKernelGGL(k_backtransform<7>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            case 8: hipLaunchKernelGGL(k_backtransform<8>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
            default: hipLaunchKernelGGL(k_backtransform<kMaxN / kWave>, gb, dim3(256), 0, st, s.Vh, s.tau, s.Zv, n, s.T, n); break;
        }
        CD_LAUNCH_CHECK();
    }
    // one Newton-Schulz step Y = T (3 I - T^T T)/2: inverse-iteration vectors of
    // eigenvalues further apart than the tight-cluster threshold are orthogonal
    // to about 1e-10, so one step brings the defect to rounding level
    const unsigned gnn = (unsigned)ceil_div((int64_t)n * n, 256);
    {
        Seg2 stt;
        stt.X1 = s.T;
        stt.ld1 = n;
        stt.p1 = n;
        CD_TRY(gram(stt, s.T, n, n, n, s.Bm, n, s.part, st, true));
        CD_TRY(update(stt, s.Bm, n, 1.0, 0.0, Y, ldy, n, n, st));
    }
    hipLaunchKernelGGL(k_copy_vec, dim3(g64), dim3(64), 0, st, s.w, evals, n);
    CD_LAUNCH_CHECK();
    return CHEBDAV_OK;
}

}  // namespace chebdav
