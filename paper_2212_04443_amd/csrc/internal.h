// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/chebdav.h"

namespace chebdav {

void set_error(const char *fmt, ...);
void clear_error();

// Returns a status after recording a message; used as `return fail(...)`.
chebdav_status fail(chebdav_status st, const char *fmt, ...);

#define CD_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::chebdav::fail(CHEBDAV_EHIP, "%s failed: %s (%s:%d)", #call,        \
                                   hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

#define CD_TRY(expr)                                                                    \
    do {                                                                                \
        chebdav_status s_ = (expr);                                                     \
        if (s_ != CHEBDAV_OK) return s_;                                                \
    } while (0)

#define CD_LAUNCH_CHECK() CD_HIP(hipGetLastError())

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device CSR pattern of S plus the degree scaling (owned by the handle).
struct Graph {
    int64_t n = 0;
    int64_t nnz = 0;
    int64_t n_isolated = 0;
    int32_t max_deg = 0;
    int64_t *row_ptr = nullptr;  // [n+1]
    int32_t *col = nullptr;      // [nnz]
    int32_t *deg = nullptr;      // [n]
    double *dinv = nullptr;      // [n]
    float *dinv32 = nullptr;     // [n], dinv rounded to FP32 (for the FP32 filter)
    double *nval = nullptr;      // [nnz], dinv of each nonzero's column (streamed by the plain product)
    // Row ranges of the sparse step per XCD: XCD x owns rows [xcd_row[x], xcd_row[x+1]),
    // chosen so that nnz + 4 * rows is about equal across the eight XCDs.
    int64_t xcd_row[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
};

// Kernel-argument copy of Graph::xcd_row.
struct XcdRanges {
    int64_t b[9];
};

// Simple bump allocator over a caller-provided workspace.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    bool counting = false;  // when true, only measures (base may be null)
    template <class T>
    T *take(size_t count) {
        used = align_up(used, 256);
        T *p = counting ? nullptr : reinterpret_cast<T *>(base + used);
        used += count * sizeof(T);
        return p;
    }
    bool overflow() const { return !counting && used > cap; }
};

// ---- csr_build.hip
chebdav_status build_graph(const int64_t *edges, int64_t n_edges, int64_t n, int on_device,
                           hipStream_t st, Graph **out);
void free_graph(Graph *g);
chebdav_status dinv_table(const int32_t *deg, double *dinv, int64_t n, hipStream_t st);

// ---- spmm.hip: Y = alpha * dinv .* (S (dinv .* U)) + beta U + gamma Z
// T = element type of U and Z (and the arithmetic), TO = element type of Y.
// Flags of the fused sparse step.  kStepScaled: U and Z hold s .* U (s = dinv,
// 1 on isolated rows), the neighbour rows are summed unscaled and the row sum
// takes dinv_i^2.  kStepOutMulS / kStepOutDivS: output times / divided by s_i.
// kStepZMulS: Z is unscaled and is multiplied by s_i.
constexpr int kStepOutMulS = 1, kStepOutDivS = 2, kStepZMulS = 4, kStepScaled = 8;
template <typename T, typename TO>
chebdav_status launch_cheb_step(const Graph *g, double alpha, double beta, double gamma,
                                const T *U, int64_t ldu, const T *Z, int64_t ldz, TO *Y,
                                int64_t ldy, int w, hipStream_t st, int flags = 0);

// Filter driver (Alg. 3); workspace laid out by filter_layout.  x_scaled: X holds
// s .* X0 (s = dinv, 1 on isolated rows) for the block X0 to be filtered; Y is
// always the filtered X0 itself.
size_t filter_ws_bytes(int64_t n, int kb, chebdav_dtype dt);
chebdav_status run_filter(const Graph *g, const double *X, int64_t ldx, double *Y, int64_t ldy,
                          int kb, int m, double cut, double upper, double scale_pt,
                          chebdav_dtype dt, void *ws, size_t ws_bytes, hipStream_t st,
                          hipEvent_t ev_begin, hipEvent_t ev_end, bool x_scaled = false);

// ---- dense.hip
// A column-segmented tall matrix: columns [0, p1) from X1 (ld1), [p1, p1+p2) from X2 (ld2).
struct Seg2 {
    const double *X1 = nullptr;
    int64_t ld1 = 0;
    int p1 = 0;
    const double *X2 = nullptr;
    int64_t ld2 = 0;
    int p2 = 0;
    __host__ __device__ int cols() const { return p1 + p2; }
};

// C (p x q, row-major, ldc) = Xs^T Y over n rows; Y: n x q (ldy).  Uses a
// deterministic split over rows with partials in `partial` (gram_partial_elems).
// With ns = true (p == q, Y = Xs) C receives (3 I - Xs^T Xs) / 2 instead: the
// matrix of one Newton-Schulz orthonormalization step X <- X C.
size_t gram_partial_elems(int64_t n, int p, int q);
chebdav_status gram(const Seg2 &Xs, const double *Y, int64_t ldy, int q, int64_t n, double *C,
                    int64_t ldc, double *partial, hipStream_t st, bool ns = false);

// Y (n x q, ldy) = alpha * Xs B + beta * Y, with B (p x q, row-major, ldb).  Y may
// alias a column block of Xs only when q <= update_max_inplace_cols().
int update_max_inplace_cols();
chebdav_status update(const Seg2 &Xs, const double *B, int64_t ldb, double alpha, double beta,
                      double *Y, int64_t ldy, int q, int64_t n, hipStream_t st);

// out[j] = ||X(:, j) - (Y ? Y(:, j) * theta[j] : 0)||_2 for j < w (n rows).
size_t colnorm_partial_elems(int64_t n, int w);
chebdav_status colnorms(const double *X, int64_t ldx, const double *Y, int64_t ldy,
                        const double *theta, int w, int64_t n, double *out, double *partial,
                        hipStream_t st);

// Row scaling applied by the block producers below when rs is not null: row r is
// multiplied by rs[r], or by 1 where rs[r] is 0 (s = dinv with 1 on isolated rows).
// Dst(:, j) = Src(:, map[j]) for j < w, row by row (Dst may equal Src: in-place
// permutation/compaction is safe because each row is staged first).  map on device.
chebdav_status gather_cols(const double *Src, int64_t lds, double *Dst, int64_t ldd,
                           const int32_t *map, int w, int64_t n, hipStream_t st, const double *rs = nullptr);
// Dst (n x w, ldd) = Src (n x w, lds), element type conversion allowed.
template <typename TS, typename TD>
chebdav_status copy_block(const TS *Src, int64_t lds, TD *Dst, int64_t ldd, int w, int64_t n,
                          hipStream_t st, const double *rs = nullptr);
// Fill a device array with a value.
chebdav_status fill_f64(double *p, int64_t count, double v, hipStream_t st);
// Philox fill (see chebdav_philox_fill).
chebdav_status philox_fill(double *X, int64_t n, int w, int64_t ld, uint64_t seed,
                           uint64_t first_col, hipStream_t st, const double *rs = nullptr);
// flag[0] |= any non-finite entry in X (n x w, ld).
// Random whole-row gathers (measurement utility); `out` holds probe_gather_out_len() doubles.
chebdav_status probe_gather(const void *table, int64_t rows, int row_bytes, int64_t gathers, uint64_t seed,
                            double *out, int64_t *performed, hipStream_t st);
int64_t probe_gather_out_len();
chebdav_status check_finite(const double *X, int64_t ld, int w, int64_t n, int *flag,
                            hipStream_t st);

// ---- small.hip (one-workgroup kernels on small matrices)
// Orthonormalization helper: from G = X^T X (kb x kb) and norm0 (pre-projection
// column norms) compute Rinv (kb x kb upper triangular) with X Rinv orthonormal,
// dep[j] = 1 for dependent columns.  scaled=1 performs the column scaling and
// dependence tests; scaled=0 is a plain Cholesky (flags a breakdown in dep[kb]).
chebdav_status chol_rinv(const double *G, int kb, const double *norm0, double *Rinv, int *dep,
                         int scaled, hipStream_t st);
// H(0:k, k-kb:k) = C (k x kb), mirrored into rows; new diagonal block symmetrized.
chebdav_status h_insert(double *H, int64_t ldh, const double *C, int k, int kb, hipStream_t st);
// H(0:k, 0:k) = diag(d).
chebdav_status h_set_diag(double *H, int64_t ldh, const double *d, int k, hipStream_t st);
// Deferred rotation (active block = B Q): H columns from Cf = [B, X]^T A X, and
// Q <- [[Q, 0], [0, I]] Y.
chebdav_status proj_cols(const double *Q, int64_t ldq, const double *Cf, int kr, int ka, int kb, double *C,
                         hipStream_t st);
chebdav_status extend_basis(const double *Q, int64_t ldq, const double *Y, int64_t ldy, int kr, int ka, int kb,
                            int nc, double *Qn, int64_t ldn, hipStream_t st);

// ---- eig.hip
size_t eig_ws_bytes(int n);
chebdav_status small_eig(const double *H, int64_t ldh, int n, double *evals, double *Y,
                         int64_t ldy, void *ws, size_t ws_bytes, hipStream_t st);

// ---- orth.hip
size_t orth_ws_bytes(int64_t n, int ksub, int kb, chebdav_orth method = CHEBDAV_ORTH_CHOLQR);
chebdav_status orthonormalize(const Seg2 &V, double *X, int64_t ldx, int kb, int64_t n,
                              uint64_t seed, uint64_t *next_col, int *n_replaced, void *ws,
                              size_t ws_bytes, hipStream_t st, chebdav_orth method = CHEBDAV_ORTH_CHOLQR);

// ---- tsqr.hip (Householder TSQR)
chebdav_status tsqr_ws_bytes(int64_t n, int kb, size_t *bytes);
// Reflectors of the leaf level to Vleaf (ldv; may be X with the same ld), the
// rest to ws; R (ldr, may be null) gets the R factor with a non-negative diagonal.
chebdav_status tsqr_factor(const double *X, int64_t ldx, int64_t n, int kb, double *Vleaf, int64_t ldv, double *R,
                           int64_t ldr, void *ws, size_t ws_bytes, hipStream_t st);
// Q (ldq; may be Vleaf with the same ld) from the reflectors of tsqr_factor.
chebdav_status tsqr_form_q(int64_t n, int kb, const double *Vleaf, int64_t ldv, double *Q, int64_t ldq, void *ws,
                           size_t ws_bytes, hipStream_t st);
chebdav_status tsqr_dep(const double *R, int64_t ldr, int kb, const double *norm0, int *dep, hipStream_t st);

// ---- gcn.hip (learned warm start)
size_t gcn_ws_bytes(int64_t n, const int dims[4]);
chebdav_status gcn_forward(const Graph *g, const int dims[4], const float *X0, const float *const W[3], float *acts,
                           float *out, void *ws, size_t ws_bytes, hipStream_t st);
chebdav_status gcn_backward(const Graph *g, const int dims[4], const float *X0, const float *const W[3],
                            const float *acts, const float *d_out, float *const dW[3], void *ws, size_t ws_bytes,
                            hipStream_t st);
chebdav_status gcn_features(const Graph *g, uint64_t seed, int n_gauss, float *X, int64_t ldx, hipStream_t st);
size_t loss_ws_bytes(int64_t n, int kx, int ku);
chebdav_status subspace_loss(const float *X, int64_t ldx, const double *U, int64_t ldu, int64_t n, int kx, int ku,
                             double *loss_host, float *dX, int64_t lddx, void *ws, size_t ws_bytes, hipStream_t st);
chebdav_status adam_step(float *w, const float *g, float *m, float *v, int64_t count, double lr, double b1,
                         double b2, double eps, int step, hipStream_t st);
chebdav_status lanczos_ws_bytes(int64_t n, int steps, size_t *bytes);
chebdav_status lanczos_bounds(const Graph *g, int steps, uint64_t seed, double *lower, double *upper,
                              double *alpha_out, double *beta_out, int *steps_done, void *ws, size_t ws_bytes,
                              hipStream_t st);
chebdav_status cluster_ws_bytes(int64_t n, int k, int K, size_t *bytes);
chebdav_status cluster(const double *U, int64_t ldu, int64_t n, int k, int K, int max_iter, uint64_t seed,
                       int32_t *labels, double *centres, int *rounds, double *inertia, void *ws, size_t ws_bytes,
                       hipStream_t st);
size_t rr_ws_bytes(int64_t n, int k);
chebdav_status rayleigh_ritz(const Graph *g, const float *X, int64_t ldx, int k, uint64_t seed, double *V,
                             int64_t ldv, double *ritz, void *ws, size_t ws_bytes, hipStream_t st);

}  // namespace chebdav
