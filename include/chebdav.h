/*
 * chebdav.h -- block Chebyshev-Davidson for the k smallest eigenpairs of the
 * normalized graph Laplacian A = I - D^{-1/2} S D^{-1/2} (Pang & Yang,
 * "A Distributed Block Chebyshev-Davidson Algorithm for Parallel Spectral
 * Clustering", arXiv 2212.04443), on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *   - Every function returns a chebdav_status; 0 is success, negative values
 *     are errors.  Nothing throws or aborts.  chebdav_last_error() returns a
 *     message for the calling thread's most recent error.
 *   - Dense blocks are ROW-MAJOR: element (i, j) of an n x w block with leading
 *     dimension ld lives at p[i * ld + j]; ld >= w.
 *   - Pointers documented as "device" must be device memory on the current HIP
 *     device; the caller owns every buffer it passes (inputs, outputs,
 *     workspaces) and keeps it alive until the stream work completes.
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream).  All work
 *     is enqueued on it in order.  Functions that must read a result back (the
 *     graph build, orthonormalize, solve) synchronize that stream before they
 *     return; chebdav_spmm and chebdav_filter do not.
 *   - On error the contents of output buffers are unspecified; nothing leaks.
 *   - Threads: a graph handle is read-only after chebdav_build_laplacian and may
 *     be shared.  Calls from different host threads, each on its own stream with
 *     its own workspace and outputs, may run concurrently: the library keeps no
 *     mutable global state (its small pinned host scratch and the error text are
 *     per thread).  Results do not depend on the interleaving.
 */
#ifndef CHEBDAV_H
#define CHEBDAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CHEBDAV_OK = 0,
    CHEBDAV_EINVAL = -1,       /* invalid argument (sizes, ids, interval, NaN input, ...) */
    CHEBDAV_ENOMEM = -2,       /* device allocation failed, workspace NULL or too small */
    CHEBDAV_EHIP = -3,         /* a HIP runtime call failed */
    CHEBDAV_ENOCONV = -4,      /* itmax reached: partial results are returned */
    CHEBDAV_EBREAKDOWN = -5,   /* no independent vector found after repeated replacement */
    CHEBDAV_EUNSUPPORTED = -6  /* a size beyond the library's limits */
} chebdav_status;

typedef enum { CHEBDAV_F64 = 0, CHEBDAV_F32 = 1 } chebdav_dtype;

/* Orthonormalization of a new block after its projections (Alg. 2 step 6):
 * Cholesky QR with a second pass (Cholesky QR or a Newton-Schulz step), or
 * Householder TSQR (Sec. 3.3). */
typedef enum { CHEBDAV_ORTH_CHOLQR = 0, CHEBDAV_ORTH_TSQR = 1 } chebdav_orth;

/* Opaque handle owning the device CSR pattern of S and its degree scaling. */
typedef struct chebdav_graph chebdav_graph;

/* ------------------------------------------------------------------------
 * Graph -> Laplacian (Eq. 1).
 *
 * Builds the canonical symmetric CSR of the simple graph: self-loops are
 * dropped, repeated edges (either orientation) merged, columns ascending in
 * each row.  deg_i = row length; dinv_i = 1/sqrt(deg_i) with IEEE
 * round-to-nearest sqrt and division, 0 for an isolated node (whose row of A is
 * the identity row, eigenvalue 1).  S is binary, so no values are stored.
 *
 * edges: n_edges x 2 int64 node ids in [0, n_nodes), 0-based, either
 * orientation; host memory if edges_on_device == 0, else device memory.
 * Errors: EINVAL for n_nodes < 1 or > 2^31 - 1, n_edges < 0 or > 2^30, or any
 * id outside [0, n_nodes) (checked on the device).
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_build_laplacian(const int64_t *edges, int64_t n_edges, int64_t n_nodes,
                                       int edges_on_device, void *hip_stream,
                                       chebdav_graph **out);

/* Sizes: n nodes, nnz stored entries (2 x unique undirected edges), isolated
 * nodes (deg = 0) and the largest degree.  Any output pointer may be NULL. */
chebdav_status chebdav_graph_info(const chebdav_graph *g, int64_t *n, int64_t *nnz,
                                  int64_t *n_isolated, int32_t *max_deg);

/* The row split the sparse step uses (host output): the eight XCDs of the GPU
 * own rows [bounds[x], bounds[x+1]), x = 0..7, contiguous ranges chosen at
 * build time so that nnz + 4 rows is about equal across them (the local share
 * of a 1-D row partition; Sec. 4 measures load imbalance over such shares). */
chebdav_status chebdav_graph_row_split(const chebdav_graph *g, int64_t bounds[9]);

/* Copies the CSR into caller device buffers: row_ptr int64[n+1], col int32[nnz],
 * deg int32[n], dinv double[n].  Any pointer may be NULL (skipped). */
chebdav_status chebdav_graph_export(const chebdav_graph *g, int64_t *row_ptr, int32_t *col,
                                    int32_t *deg, double *dinv, void *hip_stream);

/* Releases the handle and its device memory; NULL is allowed. */
void chebdav_graph_free(chebdav_graph *g);

/* ------------------------------------------------------------------------
 * Fused sparse step (the building block of Alg. 3, Sec. 3.1's SpMM):
 *
 *     Y = alpha * (D^{-1/2} S D^{-1/2}) U + beta * U + gamma * Z
 *
 * so A U = U - D^{-1/2} S D^{-1/2} U is alpha = -1, beta = 1, gamma = 0.
 * U, Z, Y: device, n x w, row-major, common leading dimension ld >= w, of the
 * element type dt.  Z may be NULL when gamma == 0.  Y must not overlap U or Z.
 * Neighbour sums are taken in ascending column order in the element type (FP32
 * accumulation for CHEBDAV_F32); results are deterministic.
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_spmm(const chebdav_graph *g, double alpha, double beta, double gamma,
                            const void *U, const void *Z, void *Y, int64_t ld, int w,
                            chebdav_dtype dt, void *hip_stream);

/* ------------------------------------------------------------------------
 * Chebyshev filter (Alg. 3; closed form Eqs. 3-5):
 *
 *     Y = p_m(A) X,   p_m(x) = C_m((x - c)/e) / C_m((scale_pt - c)/e),
 *     c = (cut + upper)/2,  e = (upper - cut)/2,
 *
 * evaluated by the scaled three-term recurrence (m sparse steps).  It damps
 * [cut, upper] to at most 1/|C_m((scale_pt - c)/e)| and keeps |p_m| <= 1 on
 * [scale_pt, upper] with p_m(scale_pt) = 1.  For the normalized Laplacian
 * upper = 2 and scale_pt = 0 (Sec. 2).
 *
 * X (input) and Y (output): device double, n x kb row-major with leading
 * dimensions ldx, ldy >= kb; X is not modified and must not overlap Y.
 * dt = CHEBDAV_F64 runs the recurrence in FP64; CHEBDAV_F32 converts X to FP32,
 * runs all m steps in FP32 with FP32 accumulation and writes Y in FP64.
 * workspace: device, at least chebdav_filter_workspace_size() bytes.
 * Errors: EINVAL unless m >= 1, kb >= 1, scale_pt < cut < upper.
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_filter_workspace_size(const chebdav_graph *g, int kb, chebdav_dtype dt,
                                             size_t *bytes);
chebdav_status chebdav_filter(const chebdav_graph *g, const double *X, int64_t ldx, double *Y,
                              int64_t ldy, int kb, int m, double cut, double upper,
                              double scale_pt, chebdav_dtype dt, void *workspace,
                              size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Filter that allocates nothing, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): chebdav_filter with its work blocks in a static device buffer of
 * the library instead of a caller workspace.  Same arguments, kernels and
 * results as chebdav_filter, minus the workspace.
 * The buffer holds 64 MiB on each GPU the library runs on, until the process
 * ends; it fits n x kb up to 3 FP64 blocks (n kb <= 2,796,000 or so, each block
 * rounded up to 256 bytes) or 4 FP32 blocks.  Larger shapes: EUNSUPPORTED.
 * Every call on one GPU uses the same buffer: calls that overlap on one GPU
 * (different streams or host threads without ordering between them) race and
 * must not be issued; calls ordered on one stream are safe.  The first call on
 * a GPU looks up the buffer's device address (no allocation); later calls make
 * no runtime call beyond the kernel launches.
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_filter_noalloc(const chebdav_graph *g, const double *X, int64_t ldx, double *Y,
                                      int64_t ldy, int kb, int m, double cut, double upper,
                                      double scale_pt, chebdav_dtype dt, void *hip_stream);

/* ------------------------------------------------------------------------
 * Block orthonormalization (Alg. 2 step 6): on return X (n x kb, device double,
 * row-major, ldx) has orthonormal columns, orthogonal to the ksub orthonormal
 * columns of V (n x ksub, device double, row-major, ldv; may be NULL if
 * ksub == 0), and spans the same space as (I - V V^T) X_in when that has full
 * numerical rank.  Method: two block classical Gram-Schmidt passes against V,
 * then (method CHOLQR) Cholesky QR with a dependence test; when the smallest
 * diagonal entry of the scaled Cholesky factor R is below 0.01, or
 * ||R^{-1}||_F (a bound on the amplification ||R^{-1}||_2 of components along V)
 * exceeds 100, a third pass against V and a second Cholesky QR, otherwise one
 * Newton-Schulz step X <- X (3 I - X^T X) / 2 (R has unit columns, so
 * kappa(R) <= 8 ||R^{-1}||_2 <= 800, X^T X is within O(kappa^2 eps) of I, and
 * the step squares that deviation); or (method TSQR) the same with Householder TSQR
 * (chebdav_tsqr) in place of each Cholesky QR, its R deciding dependence with
 * the same thresholds, and no second pass unless the third projection ran.  A column whose norm after projection
 * is below 1e-10 of its norm before, or whose squared pivot in the
 * column-scaled factor is below 1e-13, is numerically dependent and replaced
 * by a Philox4x32-10 column (key = seed, counters numbered from
 * first_random_col), then everything is redone.  n_replaced (host, may be
 * NULL) receives the number of replacements.  1 <= kb <= 64.
 * Errors: EBREAKDOWN if dependence persists after 3 rounds of replacement.
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_orthonormalize_workspace_size(int64_t n, int ksub, int kb, chebdav_orth method,
                                                     size_t *bytes);
chebdav_status chebdav_orthonormalize(const double *V, int64_t ldv, int ksub, double *X,
                                      int64_t ldx, int kb, int64_t n, uint64_t seed,
                                      uint64_t first_random_col, chebdav_orth method, int *n_replaced,
                                      void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Tall-skinny QR (Sec. 3.3, distributed orthonormalization: TSQR over a tree of
 * row blocks, here the row chunks of one GPU).  X = Q R for X (n x kb, device
 * double, row-major, ldx >= kb; only read): Q (n x kb, device double,
 * row-major, ldq >= kb) with orthonormal columns, R (kb x kb, device double,
 * row-major, ldr >= kb) upper triangular with a non-negative diagonal and
 * zeros below it; for X of full column rank this is the unique thin QR.  Q may
 * be X itself (same ld); otherwise Q, R and X must not overlap.
 * Method: Householder QR of row chunks of 256..2048 rows (one workgroup each),
 * their R factors stacked and factored again up a tree of fan-in >= 4, Q formed
 * top-down from the reflectors of every level.  Stream-ordered, no host sync.
 * workspace: device, at least chebdav_tsqr_workspace_size() bytes.
 * Errors: EINVAL if n < kb or a leading dimension is below kb; EUNSUPPORTED
 * unless 1 <= kb <= 64.
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_tsqr_workspace_size(int64_t n, int kb, size_t *bytes);
chebdav_status chebdav_tsqr(const double *X, int64_t ldx, int64_t n, int kb, double *Q, int64_t ldq,
                            double *R, int64_t ldr, void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Solver (Alg. 2: block Chebyshev-Davidson with inner-outer restart and
 * progressive filtering of initial vectors).
 * ------------------------------------------------------------------------ */
/* One Davidson iteration as seen after its restart decisions (Alg. 2 steps
 * 10-16), passed to chebdav_params.log_cb: kc = pairs locked before this
 * iteration's locking; kact = active columns after the inner restart (step 10);
 * ksub = kc + kact; n_locked = pairs locked by this iteration (step 12);
 * n_unlocked = pairs the exit certificate handed back for refinement; the
 * restart flags; low_nwb = the filter cut this iteration used (step 5);
 * min/max_residual over the residual norms of step 12. */
typedef struct {
    int iteration, kc, kact, ksub, n_locked, n_unlocked, inner_restart, outer_restart, filter_f32;
    double low_nwb, min_residual, max_residual;
} chebdav_iter_record;
typedef void (*chebdav_log_fn)(const chebdav_iter_record *rec, void *user);

typedef struct {
    int k_want;             /* number of smallest eigenpairs wanted (>= 1)                */
    int kb;                 /* block size: vectors filtered and added per iteration       */
    int m;                  /* Chebyshev filter degree                                    */
    int itmax;              /* iteration cap; 0 -> 1000                                   */
    double tol;             /* converged iff ||A v - theta v||_2 <= tol (||v|| = 1); 0 -> 1e-8 */
    int act_max;            /* 0 -> max(5 kb, 30)                  (Sec. 4)                */
    int dim_max;            /* 0 -> max(act_max + 2 kb, k_want + 30)    (Sec. 4)           */
    int k_ri;               /* inner-restart size; 0 -> max(floor(act_max/2), act_max - 3 kb) */
    double upperb;          /* spectrum upper bound; 0 -> 2                                */
    double lowb;            /* spectrum lower bound (filter scale point), normally 0       */
    double low_nwb0;        /* first cut; NaN or <= lowb -> lowb + (upperb - lowb) k_want / n */
    chebdav_dtype filter_dtype;  /* F64, or F32 for the mixed-precision form              */
    double f32_switch_tol;  /* F32 form: the residual floor of FP32 filtering (0 -> 3e-7,
                               about five FP32 unit roundoffs).  The filter runs in FP64
                               from the first iteration after which (a) when the kb
                               evaluated pairs hold every open wanted pair and the largest
                               of their residuals is at most a tenth of the distance from
                               the last wanted Ritz value theta to the next cut: one more
                               FP32 iteration, which divides residuals by
                               |C_m((theta - c)/e)| but not below this floor, would not
                               lower the predicted number of FP64 iterations; (b) otherwise:
                               the smallest open residual is below this floor; (c) in any
                               case: two FP32 iterations in a row neither locked a pair
                               nor halved the smallest open residual nor the largest
                               wanted open residual.  Every other step is always FP64   */
    uint64_t seed;          /* Philox key for all random vectors                           */
    int timing;             /* nonzero: time the filter with HIP events (stats fields)     */
    chebdav_orth orth;      /* orthonormalization of new blocks (default CHOLQR)           */
    int k_ro;               /* outer-restart size cap; 0 -> dim_max - 2 kb - kc (Sec. 2);
                               > 0 -> min(k_ro, dim_max - 2 kb - kc)                       */
    int refine_sweeps;      /* exit certificate: rounds of un-lock and refinement allowed
                               before ENOCONV; 0 -> 3, < 0 -> none                          */
    double certify_tol;     /* exit certificate: a returned pair needs a fresh
                               ||A v - lambda v||_2 <= certify_tol; 0 -> tol               */
    chebdav_log_fn log_cb;  /* nullable: called on the host once per iteration           */
    void *log_user;         /* passed to log_cb unchanged                                  */
} chebdav_params;

typedef struct {
    int iterations;         /* Davidson iterations run                                    */
    int converged;          /* locked eigenpairs (>= k_want on success)                  */
    int n_spmm_filter;      /* sparse steps spent in filters                              */
    int n_spmm_filter_f32;  /* ... of which in FP32                                       */
    int n_spmm_other;       /* other sparse products (W = A V and the exit certificate)   */
    int n_random;           /* random (Philox) columns drawn                              */
    int n_replaced;         /* of which replacements of dependent vectors                 */
    double max_residual;    /* max_i ||A v_i - lambda_i v_i||_2 of the returned pairs,
                               from a fresh sparse product after convergence              */
    double t_total_ms;      /* wall time of the call                                       */
    double t_filter_ms;     /* with timing != 0: event-timed filter time (else 0)          */
    int n_filter_launches;  /* with timing != 0: filter step launches timed                */
    int used_fallback;      /* 1 if the exit certificate un-locked a pair (refinement ran) */
    int n_unlocked;         /* pairs un-locked by the exit certificate                     */
    int n_inner_restarts;   /* Alg. 2 step 10 restarts                                     */
    int n_outer_restarts;   /* Alg. 2 step 16 restarts                                     */
} chebdav_stats;

/* Device bytes needed by chebdav_solve for this graph and these parameters. */
chebdav_status chebdav_solve_workspace_size(const chebdav_graph *g, const chebdav_params *p,
                                            size_t *bytes);

/* Finds the k_want smallest eigenpairs of A.
 * V_init: device double, n x k_init row-major (ld = k_init), may be NULL; its
 *   columns are used in the given order and should be sorted by non-decreasing
 *   Rayleigh quotient (progressive filtering, Sec. 2).  NaN/Inf -> EINVAL.
 * evals: device double[k_want], ascending.
 * evecs: device double, n x k_want row-major (ld = k_want), orthonormal columns.
 * stats: host, may be NULL.
 * Convergence (Alg. 2 step 12) is tested on the residuals the iteration keeps
 * (W - V theta, W = A V maintained through the rotations).  Once k_want pairs
 * are locked, an exit certificate recomputes ||A v - lambda v||_2 for the
 * k_want smallest with a fresh sparse product; a pair above certify_tol is
 * un-locked (at most kb per round, smallest eigenvalues first) and put at the
 * front of the next block to filter, and the iteration continues in FP64 (at
 * most refine_sweeps such rounds; stats->used_fallback, stats->n_unlocked).
 * Errors: EINVAL for invalid parameters (including dim_max < k_want + 2 kb + 1,
 * k_ri > act_max - kb, dim_max > n); ENOCONV when itmax is reached or the
 * certificate still fails after refine_sweeps rounds: the pairs found are still
 * written (the smallest locked ones, ascending) and stats->converged counts
 * those whose certificate passed. */
chebdav_status chebdav_solve(const chebdav_graph *g, const chebdav_params *p,
                             const double *V_init, int k_init, double *evals, double *evecs,
                             chebdav_stats *stats, void *workspace, size_t ws_bytes,
                             void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned warm start (not in the paper): a three-layer graph-convolution
 * network whose output block, after Rayleigh-Ritz, is passed to chebdav_solve
 * as V_init (the progressive-filtering interface of Alg. 2 steps 2 and 17).
 *
 *   Z_l = Ahat (H_{l-1} W_l), H_l = ReLU(Z_l) for l = 1, 2; out = Z_3;
 *   Ahat = D^{-1/2} S D^{-1/2};  H_0 = X0.
 *
 * dims[4] = {d0, d1, d2, d3}: input width and the three layer widths (each in
 * [1, 256]).  W[l]: device float, dims[l] x dims[l+1], row-major.  X0: device
 * float n x d0.  acts: device float, caller-owned, n x (d1 + d2): H_1 then H_2,
 * written by forward and read by backward.  out / d_out: device float n x d3.
 * dW[l]: device float, same shapes as W[l] (overwritten).  All FP32; gradient
 * sums over nodes are split in a fixed way and added in FP64 (deterministic).
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_gcn_workspace_size(const chebdav_graph *g, const int dims[4], size_t *bytes);
chebdav_status chebdav_gcn_forward(const chebdav_graph *g, const int dims[4], const float *X0,
                                   const float *const W[3], float *acts, float *out, void *workspace,
                                   size_t ws_bytes, void *hip_stream);
chebdav_status chebdav_gcn_backward(const chebdav_graph *g, const int dims[4], const float *X0,
                                    const float *const W[3], const float *acts, const float *d_out,
                                    float *const dW[3], void *workspace, size_t ws_bytes,
                                    void *hip_stream);

/* Input features X (device float, n x (n_gauss + 1), leading dimension ldx):
 * n_gauss standard normal channels (Box-Muller on Philox4x32-10, key = seed,
 * counter (row, row >> 32, channel pair, 1)) and sqrt(deg_i / mean degree),
 * mean degree = nnz / n.  One kernel, stream-ordered: no workspace, no
 * allocation, no synchronization.  Errors: EINVAL (n_gauss < 0,
 * ldx < n_gauss + 1, X NULL). */
chebdav_status chebdav_gcn_features(const chebdav_graph *g, uint64_t seed, int n_gauss, float *X,
                                    int64_t ldx, void *hip_stream);

/* Rotation- and sign-invariant subspace loss against orthonormal targets U
 * (device double, n x ku, ldu):  L = 1 - tr(U^T X (X^T X)^{-1} X^T U) / ku, and
 * dL/dX (device float, n x kx, lddx; NULL to skip).  X: device float n x kx.
 * loss: host.  kx, ku <= 64.  EBREAKDOWN if X^T X is not positive definite.
 * Synchronizes the stream. */
chebdav_status chebdav_subspace_loss_workspace_size(int64_t n, int kx, int ku, size_t *bytes);
chebdav_status chebdav_subspace_loss(const float *X, int64_t ldx, const double *U, int64_t ldu,
                                     int64_t n, int kx, int ku, double *loss, float *dX,
                                     int64_t lddx, void *workspace, size_t ws_bytes,
                                     void *hip_stream);

/* One Adam step (Kingma & Ba) on count parameters (device float arrays):
 * m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * w <- w - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  step >= 1. */
chebdav_status chebdav_adam_step(float *params, const float *grads, float *m, float *v, int64_t count,
                                 double lr, double beta1, double beta2, double eps, int step,
                                 void *hip_stream);

/* Rayleigh-Ritz of span(X) (X: device float, n x k, ldx; k <= 64): X is
 * orthonormalized (as chebdav_orthonormalize, Philox key = seed), then V (device
 * double, n x k, ldv) receives the Ritz vectors of A in ascending order of
 * their Rayleigh quotients, written to ritz (device double[k]).  This is the
 * ordering progressive filtering assumes for V_init.  Synchronizes the stream. */
chebdav_status chebdav_rayleigh_ritz_workspace_size(const chebdav_graph *g, int k, size_t *bytes);
chebdav_status chebdav_rayleigh_ritz(const chebdav_graph *g, const float *X, int64_t ldx, int k,
                                     uint64_t seed, double *V, int64_t ldv, double *ritz,
                                     void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Building blocks exposed for verification.
 * ------------------------------------------------------------------------ */
/* Symmetric eigendecomposition of the n x n matrix H (device double, row-major,
 * ldh; only read): evals ascending (device double[n]); evecs (device double,
 * n x n, row-major, ldy) with orthonormal columns, column j for evals[j].
 * Method: Householder tridiagonalization, bisection, inverse iteration with
 * reorthogonalization inside clusters, back-transformation.  1 <= n <= 1024. */
chebdav_status chebdav_small_eig_workspace_size(int n, size_t *bytes);
chebdav_status chebdav_small_eig(const double *H, int64_t ldh, int n, double *evals, double *evecs,
                                 int64_t ldy, void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Spectrum bounds by Lanczos (Sec. 2: when the filter's bounds are unknown,
 * a few Lanczos steps estimate them).
 *
 * Plain Lanczos on A without reorthogonalization, from Philox column
 * 2^32 - 1 of the seed (counter (row, row >> 32, 2^32 - 1, 0), the generator of
 * chebdav_philox_fill) scaled to unit length:
 *   w = A v_j - beta_{j-1} v_{j-1}; alpha_j = v_j . w; w -= alpha_j v_j;
 *   beta_j = ||w||_2; v_{j+1} = w / beta_j,
 * for at most `steps` steps (1..256), stopping when beta_j <= 1e-12 max(1, |alpha_j|).
 * lower / upper (host) = min / max Ritz value of the tridiagonal T_k -/+ beta_k
 * (Zhou & Li, 2011); for the normalized Laplacian the analytic interval is [0, 2].
 * alpha, beta (host, nullable, `steps` entries) receive the recurrence
 * coefficients; steps_done (host, nullable) the number of steps run.
 * Synchronizes the stream after every step.  Errors: EINVAL (steps outside
 * 1..256, NULL lower/upper), ENOMEM (workspace), EBREAKDOWN (non-finite values).
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_lanczos_bounds_workspace_size(const chebdav_graph *g, int steps, size_t *bytes);
chebdav_status chebdav_lanczos_bounds(const chebdav_graph *g, int steps, uint64_t seed, double *lower,
                                      double *upper, double *alpha, double *beta, int *steps_done,
                                      void *workspace, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Clustering tail of spectral clustering (Alg. 1, steps 3-4).
 *
 * Row normalization of the eigenvector block, then Lloyd's K-means:
 *   F(i, :) = U(i, :) / ||U(i, :)||_2 (a zero row stays zero);
 *   K initial centres by farthest-first traversal: the first is row
 *   floor(u n), u = ((w1 << 32 | w0) >> 11) / 2^53 from Philox4x32-10 with
 *   counter (0, 0, 0, 1) and key (seed mod 2^32, seed >> 32), computed in
 *   integer arithmetic; each next one is the row with the largest squared
 *   distance to its nearest chosen centre (lowest row index among ties);
 *   each round labels every row with its nearest centre (lowest centre index
 *   among ties) and moves every centre to the mean of its rows (a centre with no
 *   rows stays); rounds stop when no label changes or after max_iter rounds.
 *   Squared distances are sums over the coordinates in ascending order with
 *   separately rounded subtract, multiply and add.  All sums over rows use
 *   fixed row ranges and a fixed order (deterministic results).
 *
 * U: device double, n x k, row-major, leading dimension ldu >= k; 1 <= k <= 64.
 * labels: device int32[n] (output).  centres: device double, n_clusters x k,
 * row-major, leading dimension k (output).  rounds (host, nullable): Lloyd
 * rounds run.  inertia (host, nullable): sum over rows of the squared distance
 * to the assigned centre.  1 <= n_clusters <= min(n, 256) and
 * n_clusters * (k + 1) <= 8192.  Workspace from chebdav_cluster_workspace_size.  Synchronizes the
 * stream once per round.  Errors: EINVAL (sizes, NULL buffers, max_iter < 1),
 * ENOMEM (workspace too small), EUNSUPPORTED (n_clusters * k too large).
 * ------------------------------------------------------------------------ */
chebdav_status chebdav_cluster_workspace_size(int64_t n, int k, int n_clusters, size_t *bytes);
chebdav_status chebdav_cluster(const double *U, int64_t ldu, int64_t n, int k, int n_clusters, int max_iter,
                               uint64_t seed, int32_t *labels, double *centres, int *rounds, double *inertia,
                               void *workspace, size_t ws_bytes, void *hip_stream);

/* Fills X(:, j), j < w (device double, n x w, row-major, ld), with Philox4x32-10
 * uniforms on [-1, 1): entry (r, j) uses counter (r mod 2^32, r >> 32,
 * first_col + j, 0) and key (seed mod 2^32, seed >> 32); value =
 * ((w1 << 32 | w0) >> 11) * 2^-52 - 1 for the first two output words. */
chebdav_status chebdav_philox_fill(double *X, int64_t n, int w, int64_t ld, uint64_t seed,
                                   uint64_t first_col, void *hip_stream);

/* dinv[i] = 1/sqrt(deg[i]) (0 for deg[i] <= 0) with the device arithmetic the
 * Laplacian build uses: IEEE round-to-nearest sqrt of the degree as a double,
 * then a round-to-nearest division.  deg, dinv: device arrays of n entries. */
chebdav_status chebdav_dinv(const int32_t *deg, double *dinv, int64_t n, void *hip_stream);

/* Measurement utility (not a step of the method): `gathers` reads of whole rows
 * of `row_bytes` bytes (128, 256 or 512) at uniformly random row indices of
 * `table` (device, rows x row_bytes, row-major, 16-byte aligned; the caller
 * owns it and its contents do not matter), issued with the sparse step's load
 * shape.  This is the access pattern of the sparse step (Alg. 3; Table 1's
 * O(nnz m kb) filter term) on a graph without locality whose gathered block
 * exceeds the caches, so the time of nnz such gathers over a table the size
 * of the block bounds one step from below on the GPU at hand.  The kernel
 * rounds `gathers` up to a multiple of its group count and stores that number
 * in *performed (host, may be NULL); `out` (device) receives
 * chebdav_probe_gather_out_len() doubles that keep the loads live.  Stream-
 * ordered; the caller times the launch (events on hip_stream).  EINVAL for a
 * NULL or misaligned pointer, rows < 1, gathers < 0 or another row size. */
chebdav_status chebdav_probe_gather(const void *table, int64_t rows, int row_bytes, int64_t gathers,
                                    uint64_t seed, double *out, int64_t *performed, void *hip_stream);
int64_t chebdav_probe_gather_out_len(void);

/* Message for the calling thread's most recent error (never NULL). */
const char *chebdav_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEBDAV_H */
