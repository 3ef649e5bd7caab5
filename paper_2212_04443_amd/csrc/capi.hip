// The C ABI (include/chebdav.h): argument checks, error reporting, dispatch.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

struct chebdav_graph {
    chebdav::Graph *g;
};

// Work blocks of chebdav_filter_noalloc: one copy per GPU the library runs on,
// held until the process ends, shared by every call on that GPU.  In host code
// this name is only a handle for hipGetSymbolAddress, never a device address.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace chebdav {

namespace {
thread_local std::string g_last_error = "no error";

struct PinnedSlot {
    void *p = nullptr;
    size_t cap = 0;
    ~PinnedSlot() {
        if (p) (void)hipHostFree(p);
    }
};
thread_local PinnedSlot g_pinned[4];
}  // namespace

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error = "no error"; }

chebdav_status fail(chebdav_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of the static scratch on the current GPU.
chebdav_status static_scratch(void **out) {
    int dev = -1;
    CD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CHEBDAV_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CHEBDAV_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return CHEBDAV_OK;
}

void *pinned_host(size_t bytes, int slot) {
    PinnedSlot &s = g_pinned[slot];
    if (s.cap < bytes) {
        if (s.p) (void)hipHostFree(s.p);
        s.p = nullptr;
        s.cap = 0;
        const size_t want = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&s.p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
        s.cap = want;
    }
    return s.p;
}

chebdav_status solve_workspace_size(const Graph *g, const chebdav_params *p, size_t *bytes);
chebdav_status solve(const Graph *g, const chebdav_params *p, const double *V_init, int k_init,
                     double *evals, double *evecs, chebdav_stats *stats, void *ws, size_t ws_bytes,
                     hipStream_t st);

}  // namespace chebdav

using namespace chebdav;

#define CHECK_GRAPH(gh)                                                 \
    do {                                                                \
        if (!(gh) || !(gh)->g) return fail(CHEBDAV_EINVAL, "graph is NULL"); \
    } while (0)

extern "C" {

chebdav_status chebdav_build_laplacian(const int64_t *edges, int64_t n_edges, int64_t n_nodes,
                                       int edges_on_device, void *hip_stream, chebdav_graph **out) {
    if (!out) return fail(CHEBDAV_EINVAL, "out is NULL");
    *out = nullptr;
    Graph *g = nullptr;
    CD_TRY(build_graph(edges, n_edges, n_nodes, edges_on_device, as_stream(hip_stream), &g));
    *out = new chebdav_graph{g};
    return CHEBDAV_OK;
}

chebdav_status chebdav_graph_info(const chebdav_graph *gh, int64_t *n, int64_t *nnz,
                                  int64_t *n_isolated, int32_t *max_deg) {
    CHECK_GRAPH(gh);
    if (n) *n = gh->g->n;
    if (nnz) *nnz = gh->g->nnz;
    if (n_isolated) *n_isolated = gh->g->n_isolated;
    if (max_deg) *max_deg = gh->g->max_deg;
    return CHEBDAV_OK;
}

chebdav_status chebdav_graph_row_split(const chebdav_graph *gh, int64_t bounds[9]) {
    CHECK_GRAPH(gh);
    if (!bounds) return fail(CHEBDAV_EINVAL, "bounds is NULL");
    for (int x = 0; x < 9; ++x) bounds[x] = gh->g->xcd_row[x];
    return CHEBDAV_OK;
}

chebdav_status chebdav_graph_export(const chebdav_graph *gh, int64_t *row_ptr, int32_t *col,
                                    int32_t *deg, double *dinv, void *hip_stream) {
    CHECK_GRAPH(gh);
    const Graph *g = gh->g;
    hipStream_t st = as_stream(hip_stream);
    if (row_ptr) CD_HIP(hipMemcpyAsync(row_ptr, g->row_ptr, sizeof(int64_t) * (g->n + 1), hipMemcpyDeviceToDevice, st));
    if (col && g->nnz) CD_HIP(hipMemcpyAsync(col, g->col, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToDevice, st));
    if (deg) CD_HIP(hipMemcpyAsync(deg, g->deg, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, st));
    if (dinv) CD_HIP(hipMemcpyAsync(dinv, g->dinv, sizeof(double) * g->n, hipMemcpyDeviceToDevice, st));
    return CHEBDAV_OK;
}

void chebdav_graph_free(chebdav_graph *gh) {
    if (!gh) return;
    free_graph(gh->g);
    delete gh;
}

chebdav_status chebdav_spmm(const chebdav_graph *gh, double alpha, double beta, double gamma,
                            const void *U, const void *Z, void *Y, int64_t ld, int w,
                            chebdav_dtype dt, void *hip_stream) {
    CHECK_GRAPH(gh);
    if (U == Y || (Z && Z == Y)) return fail(CHEBDAV_EINVAL, "Y must not overlap U or Z");
    hipStream_t st = as_stream(hip_stream);
    if (dt == CHEBDAV_F64)
        return launch_cheb_step<double, double>(gh->g, alpha, beta, gamma, static_cast<const double *>(U), ld,
                                                static_cast<const double *>(Z), ld, static_cast<double *>(Y), ld, w,
                                                st);
    if (dt == CHEBDAV_F32)
        return launch_cheb_step<float, float>(gh->g, alpha, beta, gamma, static_cast<const float *>(U), ld,
                                              static_cast<const float *>(Z), ld, static_cast<float *>(Y), ld, w, st);
    return fail(CHEBDAV_EINVAL, "bad dtype");
}

chebdav_status chebdav_filter_workspace_size(const chebdav_graph *gh, int kb, chebdav_dtype dt,
                                             size_t *bytes) {
    CHECK_GRAPH(gh);
    if (!bytes || kb < 1) return fail(CHEBDAV_EINVAL, "bad arguments");
    if (dt != CHEBDAV_F64 && dt != CHEBDAV_F32) return fail(CHEBDAV_EINVAL, "bad dtype");
    *bytes = filter_ws_bytes(gh->g->n, kb, dt);
    return CHEBDAV_OK;
}

chebdav_status chebdav_filter(const chebdav_graph *gh, const double *X, int64_t ldx, double *Y,
                              int64_t ldy, int kb, int m, double cut, double upper,
                              double scale_pt, chebdav_dtype dt, void *workspace,
                              size_t ws_bytes, void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!X || !Y) return fail(CHEBDAV_EINVAL, "NULL block");
    if (X == Y) return fail(CHEBDAV_EINVAL, "X and Y must not overlap");
    return run_filter(gh->g, X, ldx, Y, ldy, kb, m, cut, upper, scale_pt, dt, workspace, ws_bytes,
                      as_stream(hip_stream), nullptr, nullptr);
}

chebdav_status chebdav_orthonormalize_workspace_size(int64_t n, int ksub, int kb, chebdav_orth method,
                                                     size_t *bytes) {
    if (!bytes || n < 1 || ksub < 0 || kb < 1) return fail(CHEBDAV_EINVAL, "bad arguments");
    if (method != CHEBDAV_ORTH_CHOLQR && method != CHEBDAV_ORTH_TSQR) return fail(CHEBDAV_EINVAL, "bad method");
    if (method == CHEBDAV_ORTH_TSQR) {
        size_t tb = 0;
        CD_TRY(tsqr_ws_bytes(n, kb, &tb));
    }
    *bytes = orth_ws_bytes(n, ksub, kb, method);
    return CHEBDAV_OK;
}

chebdav_status chebdav_tsqr_workspace_size(int64_t n, int kb, size_t *bytes) {
    if (!bytes) return fail(CHEBDAV_EINVAL, "bytes is NULL");
    return tsqr_ws_bytes(n, kb, bytes);
}

chebdav_status chebdav_tsqr(const double *X, int64_t ldx, int64_t n, int kb, double *Q, int64_t ldq,
                            double *R, int64_t ldr, void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!X || !Q || !R) return fail(CHEBDAV_EINVAL, "NULL argument");
    if (Q == X && ldq != ldx) return fail(CHEBDAV_EINVAL, "Q == X needs ldq == ldx");
    hipStream_t st = as_stream(hip_stream);
    CD_TRY(tsqr_factor(X, ldx, n, kb, Q, ldq, R, ldr, workspace, ws_bytes, st));
    CD_TRY(tsqr_form_q(n, kb, Q, ldq, Q, ldq, workspace, ws_bytes, st));
    return CHEBDAV_OK;
}

chebdav_status chebdav_orthonormalize(const double *V, int64_t ldv, int ksub, double *X,
                                      int64_t ldx, int kb, int64_t n, uint64_t seed,
                                      uint64_t first_random_col, chebdav_orth method, int *n_replaced,
                                      void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!X || n < 1 || kb < 1 || ksub < 0 || ldx < kb) return fail(CHEBDAV_EINVAL, "bad arguments");
    if (ksub > 0 && (!V || ldv < ksub)) return fail(CHEBDAV_EINVAL, "bad basis V");
    Seg2 v;
    v.X1 = V;
    v.ld1 = ldv;
    v.p1 = ksub;
    uint64_t next = first_random_col;
    int rep = 0;
    hipStream_t st = as_stream(hip_stream);
    CD_TRY(orthonormalize(v, X, ldx, kb, n, seed, &next, &rep, workspace, ws_bytes, st, method));
    CD_HIP(hipStreamSynchronize(st));
    if (n_replaced) *n_replaced = rep;
    return CHEBDAV_OK;
}

chebdav_status chebdav_solve_workspace_size(const chebdav_graph *gh, const chebdav_params *p,
                                            size_t *bytes) {
    CHECK_GRAPH(gh);
    if (!bytes) return fail(CHEBDAV_EINVAL, "bytes is NULL");
    return solve_workspace_size(gh->g, p, bytes);
}

chebdav_status chebdav_solve(const chebdav_graph *gh, const chebdav_params *p,
                             const double *V_init, int k_init, double *evals, double *evecs,
                             chebdav_stats *stats, void *workspace, size_t ws_bytes,
                             void *hip_stream) {
    CHECK_GRAPH(gh);
    return solve(gh->g, p, V_init, k_init, evals, evecs, stats, workspace, ws_bytes, as_stream(hip_stream));
}

chebdav_status chebdav_small_eig_workspace_size(int n, size_t *bytes) {
    if (!bytes || n < 1 || n > 1024) return fail(CHEBDAV_EINVAL, "n must be in [1, 1024]");
    *bytes = eig_ws_bytes(n);
    return CHEBDAV_OK;
}

chebdav_status chebdav_small_eig(const double *H, int64_t ldh, int n, double *evals, double *evecs,
                                 int64_t ldy, void *workspace, size_t ws_bytes, void *hip_stream) {
    if (!H || !evals || !evecs) return fail(CHEBDAV_EINVAL, "NULL argument");
    return small_eig(H, ldh, n, evals, evecs, ldy, workspace, ws_bytes, as_stream(hip_stream));
}

chebdav_status chebdav_lanczos_bounds_workspace_size(const chebdav_graph *g, int steps, size_t *bytes) {
    CHECK_GRAPH(g);
    if (!bytes) return fail(CHEBDAV_EINVAL, "bytes is NULL");
    return lanczos_ws_bytes(g->g->n, steps, bytes);
}

chebdav_status chebdav_lanczos_bounds(const chebdav_graph *g, int steps, uint64_t seed, double *lower,
                                      double *upper, double *alpha, double *beta, int *steps_done,
                                      void *workspace, size_t ws_bytes, void *hip_stream) {
    CHECK_GRAPH(g);
    return lanczos_bounds(g->g, steps, seed, lower, upper, alpha, beta, steps_done, workspace, ws_bytes,
                          as_stream(hip_stream));
}

chebdav_status chebdav_cluster_workspace_size(int64_t n, int k, int n_clusters, size_t *bytes) {
    if (!bytes) return fail(CHEBDAV_EINVAL, "bytes is NULL");
    return cluster_ws_bytes(n, k, n_clusters, bytes);
}

chebdav_status chebdav_cluster(const double *U, int64_t ldu, int64_t n, int k, int n_clusters, int max_iter,
                               uint64_t seed, int32_t *labels, double *centres, int *rounds, double *inertia,
                               void *workspace, size_t ws_bytes, void *hip_stream) {
    return cluster(U, ldu, n, k, n_clusters, max_iter, seed, labels, centres, rounds, inertia, workspace, ws_bytes,
                   as_stream(hip_stream));
}

chebdav_status chebdav_philox_fill(double *X, int64_t n, int w, int64_t ld, uint64_t seed,
                                   uint64_t first_col, void *hip_stream) {
    if (!X || n < 0 || w < 0 || ld < w) return fail(CHEBDAV_EINVAL, "bad arguments");
    return philox_fill(X, n, w, ld, seed, first_col, as_stream(hip_stream));
}

chebdav_status chebdav_probe_gather(const void *table, int64_t rows, int row_bytes, int64_t gathers,
                                    uint64_t seed, double *out, int64_t *performed, void *hip_stream) {
    return probe_gather(table, rows, row_bytes, gathers, seed, out, performed, as_stream(hip_stream));
}

int64_t chebdav_probe_gather_out_len(void) { return probe_gather_out_len(); }

chebdav_status chebdav_dinv(const int32_t *deg, double *dinv, int64_t n, void *hip_stream) {
    if (n < 0 || (n > 0 && (!deg || !dinv))) return fail(CHEBDAV_EINVAL, "bad arguments");
    return dinv_table(deg, dinv, n, as_stream(hip_stream));
}

chebdav_status chebdav_gcn_workspace_size(const chebdav_graph *gh, const int dims[4], size_t *bytes) {
    CHECK_GRAPH(gh);
    if (!dims || !bytes) return fail(CHEBDAV_EINVAL, "NULL argument");
    *bytes = gcn_ws_bytes(gh->g->n, dims);
    return CHEBDAV_OK;
}

chebdav_status chebdav_gcn_features(const chebdav_graph *gh, uint64_t seed, int n_gauss, float *X, int64_t ldx,
                                    void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!X) return fail(CHEBDAV_EINVAL, "X is NULL");
    return gcn_features(gh->g, seed, n_gauss, X, ldx, as_stream(hip_stream));
}

chebdav_status chebdav_gcn_forward(const chebdav_graph *gh, const int dims[4], const float *X0,
                                   const float *const W[3], float *acts, float *out, void *workspace,
                                   size_t ws_bytes, void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!dims || !X0 || !W || !W[0] || !W[1] || !W[2] || !acts || !out) return fail(CHEBDAV_EINVAL, "NULL argument");
    return gcn_forward(gh->g, dims, X0, W, acts, out, workspace, ws_bytes, as_stream(hip_stream));
}

chebdav_status chebdav_gcn_backward(const chebdav_graph *gh, const int dims[4], const float *X0,
                                    const float *const W[3], const float *acts, const float *d_out,
                                    float *const dW[3], void *workspace, size_t ws_bytes, void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!dims || !X0 || !W || !acts || !d_out || !dW || !dW[0] || !dW[1] || !dW[2])
        return fail(CHEBDAV_EINVAL, "NULL argument");
    return gcn_backward(gh->g, dims, X0, W, acts, d_out, dW, workspace, ws_bytes, as_stream(hip_stream));
}

chebdav_status chebdav_subspace_loss_workspace_size(int64_t n, int kx, int ku, size_t *bytes) {
    if (!bytes || n < 1 || kx < 1 || ku < 1) return fail(CHEBDAV_EINVAL, "bad arguments");
    *bytes = loss_ws_bytes(n, kx, ku);
    return CHEBDAV_OK;
}

chebdav_status chebdav_subspace_loss(const float *X, int64_t ldx, const double *U, int64_t ldu, int64_t n, int kx,
                                     int ku, double *loss, float *dX, int64_t lddx, void *workspace,
                                     size_t ws_bytes, void *hip_stream) {
    if (!X || !U || ldx < kx || ldu < ku || (dX && lddx < kx)) return fail(CHEBDAV_EINVAL, "bad arguments");
    return subspace_loss(X, ldx, U, ldu, n, kx, ku, loss, dX, lddx, workspace, ws_bytes, as_stream(hip_stream));
}

chebdav_status chebdav_adam_step(float *params, const float *grads, float *m, float *v, int64_t count, double lr,
                                 double beta1, double beta2, double eps, int step, void *hip_stream) {
    if (count > 0 && (!params || !grads || !m || !v)) return fail(CHEBDAV_EINVAL, "NULL argument");
    return adam_step(params, grads, m, v, count, lr, beta1, beta2, eps, step, as_stream(hip_stream));
}

chebdav_status chebdav_rayleigh_ritz_workspace_size(const chebdav_graph *gh, int k, size_t *bytes) {
    CHECK_GRAPH(gh);
    if (!bytes || k < 1) return fail(CHEBDAV_EINVAL, "bad arguments");
    *bytes = rr_ws_bytes(gh->g->n, k);
    return CHEBDAV_OK;
}

chebdav_status chebdav_rayleigh_ritz(const chebdav_graph *gh, const float *X, int64_t ldx, int k, uint64_t seed,
                                     double *V, int64_t ldv, double *ritz, void *workspace, size_t ws_bytes,
                                     void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!X || !V || !ritz || ldx < k || ldv < k) return fail(CHEBDAV_EINVAL, "bad arguments");
    hipStream_t st = as_stream(hip_stream);
    CD_TRY(rayleigh_ritz(gh->g, X, ldx, k, seed, V, ldv, ritz, workspace, ws_bytes, st));
    CD_HIP(hipStreamSynchronize(st));
    return CHEBDAV_OK;
}

// Filter on the static scratch.  The device address of `scratch` is looked up
// once per GPU (with that GPU current) on the first call made there and kept.
chebdav_status chebdav_filter_noalloc(const chebdav_graph *gh, const double *X, int64_t ldx, double *Y,
                                      int64_t ldy, int kb, int m, double cut, double upper, double scale_pt,
                                      chebdav_dtype dt, void *hip_stream) {
    CHECK_GRAPH(gh);
    if (!X || !Y) return fail(CHEBDAV_EINVAL, "NULL block");
    if (X == Y) return fail(CHEBDAV_EINVAL, "X and Y must not overlap");
    if (kb < 1) return fail(CHEBDAV_EINVAL, "kb must be >= 1");
    if (dt != CHEBDAV_F64 && dt != CHEBDAV_F32) return fail(CHEBDAV_EINVAL, "bad dtype");
    const size_t need = filter_ws_bytes(gh->g->n, kb, dt);
    if (need > kStaticScratchBytes)
        return fail(CHEBDAV_EUNSUPPORTED,
                    "chebdav_filter_noalloc: %lld x %d needs %zu bytes of work blocks, more than the %zu-byte "
                    "static scratch (use chebdav_filter with a workspace)",
                    (long long)gh->g->n, kb, need, kStaticScratchBytes);
    void *ws = nullptr;
    CD_TRY(static_scratch(&ws));
    return run_filter(gh->g, X, ldx, Y, ldy, kb, m, cut, upper, scale_pt, dt, ws, kStaticScratchBytes,
                      as_stream(hip_stream), nullptr, nullptr);
}

const char *chebdav_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
