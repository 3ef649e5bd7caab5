// Block orthonormalization of a new block X against the basis V (Alg. 2 step 6).
//
// Sec. 2 orthonormalizes with DGKS, replacing numerically dependent vectors by
// random ones.  Column-by-column Gram-Schmidt is a chain of matrix-vector
// products; here the same result (an orthonormal basis of span((I - V V^T) X)
// that is orthogonal to V) is reached with block operations that run as
// matrix-matrix products over all of X:
//   BCGS2     X <- X - V (V^T X), twice (classical Gram-Schmidt + reorthogonalization)
//   CholQR    G = X^T X; the columns are scaled to unit norm and G = R^T R;
//             X <- X S R^{-1}.  A column is dependent when its norm after
//             projection is below 1e-10 of its norm before (the threshold the
//             DGKS reading uses) or its pivot in the scaled Gram matrix is below
//             1e-13 (then it lies, to working accuracy, in the span of the
//             columns before it).  Dependent columns are replaced by Philox
//             columns and everything is redone.
//   BCGS      one more pass against V when the smallest scaled pivot is below
//             0.01 or ||R^{-1}||_F of the scaled factor (a bound on its
//             ||R^{-1}||_2) exceeds 100 (R^{-1} may then amplify the
//             remaining non-orthogonality to V above rounding level), then a
//             second, plain CholQR; otherwise one Newton-Schulz step
//             X <- X (3 I - X^T X) / 2 in its place.
// With CHEBDAV_ORTH_TSQR the two Cholesky QRs are replaced by Householder TSQR
// (Sec. 3.3): R of the projected block decides dependence with the same
// thresholds (column norms from R's columns, scaled pivots R_jj / ||R(:, j)||),
// then X <- Q; the third projection is followed by a second TSQR.  TSQR needs
// no condition-number bound, at about ten times the cost of Cholesky QR.
#include <algorithm>

#include "device_util.h"
#include "internal.h"

namespace chebdav {

// Per-thread pinned host buffer used for small device-to-host reads.
void *pinned_host(size_t bytes, int slot);

namespace {

struct OrthWs {
    double *C, *G, *Rinv, *norm0, *part;
    int *dep;
    double *vleaf = nullptr;  // TSQR: reflectors of the leaf level (n x kb)
    void *tsqr = nullptr;
    size_t tsqr_b = 0;
};

OrthWs orth_layout(Arena &a, int64_t n, int ksub, int kb, chebdav_orth method) {
    OrthWs s;
    s.C = a.take<double>((size_t)std::max(ksub, 1) * kb);
    s.G = a.take<double>((size_t)kb * kb);
    s.Rinv = a.take<double>((size_t)kb * kb);
    s.norm0 = a.take<double>(kb);
    s.dep = a.take<int>(kb + 2);
    size_t pe = std::max(gram_partial_elems(n, std::max(ksub, 1), kb), gram_partial_elems(n, kb, kb));
    pe = std::max(pe, colnorm_partial_elems(n, kb));
    s.part = a.take<double>(pe);
    if (method == CHEBDAV_ORTH_TSQR) {
        s.vleaf = a.take<double>((size_t)n * kb);
        if (tsqr_ws_bytes(n, kb, &s.tsqr_b) != CHEBDAV_OK) s.tsqr_b = 0;
        s.tsqr = a.take<char>(s.tsqr_b);
    }
    return s;
}

chebdav_status project_out(const Seg2 &V, double *X, int64_t ldx, int kb, int64_t n, const OrthWs &s,
                           hipStream_t st) {
    if (V.cols() == 0) return CHEBDAV_OK;
    CD_TRY(gram(V, X, ldx, kb, n, s.C, kb, s.part, st));
    CD_TRY(update(V, s.C, kb, -1.0, 1.0, X, ldx, kb, n, st));
    return CHEBDAV_OK;
}

chebdav_status replace_dependent(const int *hdep, double *X, int64_t ldx, int kb, int64_t n, uint64_t seed,
                                 uint64_t *next_col, int *replaced, const OrthWs &s, hipStream_t st) {
    for (int j = 0; j < kb; ++j) {
        if (!hdep[j]) continue;
        CD_TRY(philox_fill(X + j, n, 1, ldx, seed, *next_col, st));
        *next_col += 1;
        ++*replaced;
        CD_TRY(colnorms(X + j, ldx, nullptr, 0, nullptr, 1, n, s.norm0 + j, s.part, st));
    }
    return CHEBDAV_OK;
}

chebdav_status orthonormalize_tsqr(const Seg2 &V, double *X, int64_t ldx, int kb, int64_t n, uint64_t seed,
                                   uint64_t *next_col, int *n_replaced, const OrthWs &s, hipStream_t st) {
    int *hdep = static_cast<int *>(pinned_host(sizeof(int) * (kb + 2), 2));
    if (!hdep) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    int replaced = 0;
    CD_TRY(colnorms(X, ldx, nullptr, 0, nullptr, kb, n, s.norm0, s.part, st));
    for (int attempt = 0;; ++attempt) {
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(tsqr_factor(X, ldx, n, kb, s.vleaf, kb, s.G, kb, s.tsqr, s.tsqr_b, st));
        CD_TRY(tsqr_dep(s.G, kb, kb, s.norm0, s.dep, st));
        CD_HIP(hipMemcpyAsync(hdep, s.dep, sizeof(int) * (kb + 2), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        if (!hdep[kb]) break;
        if (attempt == 3) return fail(CHEBDAV_EBREAKDOWN, "dependent vectors persist after 3 replacement rounds");
        CD_TRY(replace_dependent(hdep, X, ldx, kb, n, seed, next_col, &replaced, s, st));
    }
    CD_TRY(tsqr_form_q(n, kb, s.vleaf, kb, X, ldx, s.tsqr, s.tsqr_b, st));
    if (hdep[kb + 1]) {
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(tsqr_factor(X, ldx, n, kb, s.vleaf, kb, nullptr, kb, s.tsqr, s.tsqr_b, st));
        CD_TRY(tsqr_form_q(n, kb, s.vleaf, kb, X, ldx, s.tsqr, s.tsqr_b, st));
    }
    if (n_replaced) *n_replaced = replaced;
    return CHEBDAV_OK;
}

}  // namespace

size_t orth_ws_bytes(int64_t n, int ksub, int kb, chebdav_orth method) {
    Arena a;
    a.counting = true;
    (void)orth_layout(a, n, ksub, kb, method);
    return a.used + 256;
}

chebdav_status orthonormalize(const Seg2 &V, double *X, int64_t ldx, int kb, int64_t n,
                              uint64_t seed, uint64_t *next_col, int *n_replaced, void *ws,
                              size_t ws_bytes, hipStream_t st, chebdav_orth method) {
    if (kb < 1 || kb > update_max_inplace_cols()) return fail(CHEBDAV_EUNSUPPORTED, "kb must be in [1, %d]", update_max_inplace_cols());
    if (n < (int64_t)V.cols() + kb) return fail(CHEBDAV_EINVAL, "n < ksub + kb: no room for an orthonormal block");
    if (method != CHEBDAV_ORTH_CHOLQR && method != CHEBDAV_ORTH_TSQR) return fail(CHEBDAV_EINVAL, "bad orthonormalization method");
    if (method == CHEBDAV_ORTH_TSQR) {
        size_t tb = 0;
        CD_TRY(tsqr_ws_bytes(n, kb, &tb));
    }
    const size_t need = orth_ws_bytes(n, V.cols(), kb, method);
    if (!ws || ws_bytes < need) return fail(CHEBDAV_ENOMEM, "orthonormalize workspace too small (%zu < %zu)", ws_bytes, need);
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const OrthWs s = orth_layout(a, n, V.cols(), kb, method);
    if (method == CHEBDAV_ORTH_TSQR) return orthonormalize_tsqr(V, X, ldx, kb, n, seed, next_col, n_replaced, s, st);
    int *hdep = static_cast<int *>(pinned_host(sizeof(int) * (kb + 2), 2));
    if (!hdep) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    Seg2 xs;
    xs.X1 = X;
    xs.ld1 = ldx;
    xs.p1 = kb;
    int replaced = 0;
    CD_TRY(colnorms(X, ldx, nullptr, 0, nullptr, kb, n, s.norm0, s.part, st));
    for (int attempt = 0;; ++attempt) {
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(gram(xs, X, ldx, kb, n, s.G, kb, s.part, st));
        CD_TRY(chol_rinv(s.G, kb, s.norm0, s.Rinv, s.dep, 1, st));
        CD_HIP(hipMemcpyAsync(hdep, s.dep, sizeof(int) * (kb + 2), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        if (!hdep[kb]) break;
        if (attempt == 3) return fail(CHEBDAV_EBREAKDOWN, "dependent vectors persist after 3 replacement rounds");
        CD_TRY(replace_dependent(hdep, X, ldx, kb, n, seed, next_col, &replaced, s, st));
    }
    CD_TRY(update(xs, s.Rinv, kb, 1.0, 0.0, X, ldx, kb, n, st));
    // a third projection only when R^{-1} can have amplified the remaining
    // components along V above rounding level (smallest scaled pivot < 0.01, or
    // ||R^{-1}||_F of the scaled factor above 100); then a second Cholesky QR.
    // Otherwise the first Cholesky QR left X^T X within O(kappa^2 eps) of I with
    // kappa <= 8 ||R^{-1}||_2 <= 800 (unit columns, kb <= 64), and one
    // Newton-Schulz step X (3 I - X^T X) / 2 squares that deviation.
    if (hdep[kb + 1]) {
        CD_TRY(project_out(V, X, ldx, kb, n, s, st));
        CD_TRY(gram(xs, X, ldx, kb, n, s.G, kb, s.part, st));
        CD_TRY(chol_rinv(s.G, kb, nullptr, s.Rinv, s.dep, 0, st));
    } else {
        CD_TRY(gram(xs, X, ldx, kb, n, s.Rinv, kb, s.part, st, true));
    }
    CD_TRY(update(xs, s.Rinv, kb, 1.0, 0.0, X, ldx, kb, n, st));
    if (n_replaced) *n_replaced = replaced;
    return CHEBDAV_OK;
}

}  // namespace chebdav
