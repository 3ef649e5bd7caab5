// Host driver of block Chebyshev-Davidson with inner-outer restart (Alg. 2).
//
// Every step runs on the device; the host keeps only the integer bookkeeping
// (kc, kact, ksub, ki), the Ritz values of the active block and the residual
// norms of its first kb pairs, read back once per iteration (step 12).
//
// Readings of what the algorithm leaves open (shared with the CPU oracle):
// ascending Ritz order everywhere; filter interval cut = low_nwb, upper =
// upperb, scale point = lowb, first cut lowb + (upperb - lowb) k_want / n;
// convergence ||W(:,i) - V(:,kc+i) theta_i||_2 <= tol; every converged pair
// among the first kb is locked; low_nwb = median of the kact retained Ritz
// values (mean of the middle two for an even count), kept if not strictly
// inside (lowb, upperb); missing vectors are Philox columns numbered in the
// order they are drawn; k_ri = max(floor(act_max/2), act_max - 3 kb),
// k_ro = dim_max - 2 kb - kc, act_max = max(5 kb, 30),
// dim_max = max(act_max + 2 kb, k_want + 30).
//
// Device layout (all row-major):
//   Vl    n x (k_want + kb)   locked Ritz vectors, in locking order
//   Va[2] n x act_max         active block V(:, kc+1 : ksub), double-buffered so
//                             the rotation V <- V Y writes out of place
//   W[2]  n x act_max         W = A V for the active block, double-buffered
//   Vtmp  n x kb              s .* (the block to filter next), s = dinv (1 on isolated rows)
// V(:, 1:ksub) of the algorithm is the pair [Vl(:, 1:kc), Va(:, 1:kact)]; the
// locked set is sorted by eigenvalue only when the result is written.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace chebdav {

void *pinned_host(size_t bytes, int slot);

namespace {

struct Resolved {
    int k_want, kb, m, itmax, act_max, dim_max, k_ri, k_ro, refine_sweeps, lmax;
    double tol, certify_tol, upperb, lowb, low_nwb0, f32_switch_tol;
    chebdav_dtype fdt;
    chebdav_orth orth;
    uint64_t seed;
    bool timing;
    chebdav_log_fn log_cb;
    void *log_user;
    // size of the active block after an outer restart (step 16) with kc locked
    int ro_size(int kc) const {
        const int k = dim_max - 2 * kb - kc;
        return k_ro > 0 ? std::min(k_ro, k) : k;
    }
};

chebdav_status resolve(const chebdav_params *p, int64_t n, Resolved &r) {
    if (!p) return fail(CHEBDAV_EINVAL, "params is NULL");
    r.k_want = p->k_want;
    r.kb = p->kb;
    r.m = p->m;
    r.itmax = p->itmax > 0 ? p->itmax : 1000;
    r.tol = p->tol > 0 ? p->tol : 1e-8;
    r.certify_tol = p->certify_tol > 0 ? p->certify_tol : r.tol;
    r.k_ro = p->k_ro;
    r.refine_sweeps = p->refine_sweeps == 0 ? 3 : std::max(0, p->refine_sweeps);
    r.log_cb = p->log_cb;
    r.log_user = p->log_user;
    r.act_max = p->act_max > 0 ? p->act_max : std::max(5 * r.kb, 30);
    r.dim_max = p->dim_max > 0 ? p->dim_max : std::max(r.act_max + 2 * r.kb, r.k_want + 30);
    r.k_ri = p->k_ri > 0 ? p->k_ri : std::max(r.act_max / 2, r.act_max - 3 * r.kb);
    r.upperb = p->upperb != 0.0 ? p->upperb : 2.0;
    r.lowb = p->lowb;
    r.low_nwb0 = (std::isnan(p->low_nwb0) || p->low_nwb0 <= r.lowb)
                     ? r.lowb + (r.upperb - r.lowb) * r.k_want / (double)n
                     : p->low_nwb0;
    r.f32_switch_tol = p->f32_switch_tol > 0 ? p->f32_switch_tol : 3e-7;
    r.fdt = p->filter_dtype;
    r.orth = p->orth;
    r.seed = p->seed;
    r.timing = p->timing != 0;
    r.lmax = r.k_want + r.kb;
    if (r.kb < 1 || r.k_want < 1 || r.m < 1) return fail(CHEBDAV_EINVAL, "need kb >= 1, k_want >= 1, m >= 1");
    if (!(r.tol > 0) || !(r.certify_tol > 0) || std::isnan(p->certify_tol) || std::isnan(p->tol))
        return fail(CHEBDAV_EINVAL, "tolerances must be positive numbers");
    if (r.k_ro < 0) return fail(CHEBDAV_EINVAL, "k_ro < 0");
    if (r.k_want > n) return fail(CHEBDAV_EINVAL, "k_want > n");
    if (r.kb > update_max_inplace_cols()) return fail(CHEBDAV_EUNSUPPORTED, "kb > %d", update_max_inplace_cols());
    if (r.k_ri < 1 || r.k_ri > r.act_max - r.kb) return fail(CHEBDAV_EINVAL, "need 1 <= k_ri <= act_max - kb");
    if (r.dim_max < r.k_want + 2 * r.kb + 1 || r.dim_max < r.act_max)
        return fail(CHEBDAV_EINVAL, "need dim_max >= max(k_want + 2 kb + 1, act_max)");
    if (r.dim_max > n) return fail(CHEBDAV_EINVAL, "dim_max > n");
    if (r.act_max > 512) return fail(CHEBDAV_EUNSUPPORTED, "act_max > 512");
    if (!(r.lowb < r.low_nwb0 && r.low_nwb0 < r.upperb)) return fail(CHEBDAV_EINVAL, "need lowb < low_nwb0 < upperb");
    if (r.fdt != CHEBDAV_F64 && r.fdt != CHEBDAV_F32) return fail(CHEBDAV_EINVAL, "bad filter dtype");
    if (r.orth != CHEBDAV_ORTH_CHOLQR && r.orth != CHEBDAV_ORTH_TSQR) return fail(CHEBDAV_EINVAL, "bad orth method");
    if (r.orth == CHEBDAV_ORTH_TSQR && r.kb > 64) return fail(CHEBDAV_EUNSUPPORTED, "TSQR needs kb <= 64");
    return CHEBDAV_OK;
}

struct Layout {
    double *Vl, *Va[2], *W[2], *Vtmp, *H, *C, *C2, *Y, *Q[2], *D, *res, *part, *hd, *ev, *ones;
    int32_t *map;
    void *filt, *orthw, *eigw;
    size_t filt_b, orth_b, eig_b;
};

// Index-map regions (int32), the same on the device and in the pinned host
// buffer: converged / retained active columns (act_max each), then the exit
// certificate's order, the columns it un-locks and the locked columns it keeps
// (k_want + kb each).
size_t map_entries(const Resolved &r) { return (size_t)2 * r.act_max + 3 * r.lmax; }
size_t map_cert(const Resolved &r) { return (size_t)2 * r.act_max; }
size_t map_unl(const Resolved &r) { return (size_t)2 * r.act_max + r.lmax; }
size_t map_keep(const Resolved &r) { return (size_t)2 * r.act_max + 2 * r.lmax; }

Layout layout(Arena &a, int64_t n, const Resolved &r) {
    Layout L;
    L.Vl = a.take<double>((size_t)n * r.lmax);
    for (int i = 0; i < 2; ++i) L.Va[i] = a.take<double>((size_t)n * r.act_max);
    for (int i = 0; i < 2; ++i) L.W[i] = a.take<double>((size_t)n * r.act_max);
    L.Vtmp = a.take<double>((size_t)n * r.kb);
    L.H = a.take<double>((size_t)r.act_max * r.act_max);
    L.C = a.take<double>((size_t)r.act_max * r.kb);
    L.C2 = a.take<double>((size_t)r.act_max * r.kb);
    L.Y = a.take<double>((size_t)r.act_max * r.act_max);
    for (int i = 0; i < 2; ++i) L.Q[i] = a.take<double>((size_t)r.act_max * r.act_max);
    L.ones = a.take<double>(r.act_max);
    // Ritz values and residual norms side by side (one device-to-host copy)
    L.D = a.take<double>((size_t)r.act_max + std::max(r.act_max, r.lmax));
    L.res = L.D + r.act_max;
    L.ev = a.take<double>(r.lmax);
    size_t pe = std::max(gram_partial_elems(n, r.act_max, r.kb), colnorm_partial_elems(n, std::min(256, std::max(r.act_max, r.kb))));
    L.part = a.take<double>(pe);
    // index maps followed by the new diagonal of H, laid out as in the pinned
    // host buffer (one host-to-device copy per iteration)
    {
        const size_t nm = map_entries(r);
        char *mh = a.take<char>(sizeof(int32_t) * nm + sizeof(double) * (r.act_max + r.lmax));
        L.map = reinterpret_cast<int32_t *>(mh);
        L.hd = reinterpret_cast<double *>(mh + sizeof(int32_t) * nm);
    }
    L.filt_b = std::max(filter_ws_bytes(n, r.kb, CHEBDAV_F64),
                        r.fdt == CHEBDAV_F32 ? filter_ws_bytes(n, r.kb, CHEBDAV_F32) : 0);
    L.filt = a.take<char>(L.filt_b);
    L.orth_b = orth_ws_bytes(n, r.dim_max, r.kb, r.orth);
    L.orthw = a.take<char>(L.orth_b);
    L.eig_b = eig_ws_bytes(r.act_max);
    L.eigw = a.take<char>(L.eig_b);
    return L;
}

double median_of(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t h = v.size() / 2;
    return v.size() % 2 ? v[h] : 0.5 * (v[h - 1] + v[h]);
}

struct EventPair {
    hipEvent_t b = nullptr, e = nullptr;
    ~EventPair() {
        if (b) (void)hipEventDestroy(b);
        if (e) (void)hipEventDestroy(e);
    }
};

}  // namespace

chebdav_status solve_workspace_size(const Graph *g, const chebdav_params *p, size_t *bytes) {
    Resolved r;
    CD_TRY(resolve(p, g->n, r));
    Arena a;
    a.counting = true;
    (void)layout(a, g->n, r);
    *bytes = a.used + 256;
    return CHEBDAV_OK;
}

chebdav_status solve(const Graph *g, const chebdav_params *p, const double *V_init, int k_init,
                     double *evals, double *evecs, chebdav_stats *stats, void *ws, size_t ws_bytes,
                     hipStream_t st) {
    const auto t_start = std::chrono::steady_clock::now();
    Resolved r;
    CD_TRY(resolve(p, g->n, r));
    const int64_t n = g->n;
    const int kb = r.kb, am = r.act_max;
    if (k_init < 0 || (k_init > 0 && !V_init)) return fail(CHEBDAV_EINVAL, "bad V_init / k_init");
    if (!evals || !evecs) return fail(CHEBDAV_EINVAL, "evals/evecs are NULL");
    {
        Arena c;
        c.counting = true;
        (void)layout(c, n, r);
        if (!ws || ws_bytes < c.used + 256)
            return fail(CHEBDAV_ENOMEM, "solve workspace too small (%zu < %zu)", ws_bytes, c.used + 256);
    }
    Arena a;
    a.base = static_cast<char *>(ws);
    a.cap = ws_bytes;
    const Layout L = layout(a, n, r);

    // pinned host scratch: [0] Ritz values + residuals, [1] index maps / diagonal
    double *h_vals = static_cast<double *>(pinned_host(sizeof(double) * (2 * am + 2 * r.lmax + 8), 0));
    int32_t *h_map = static_cast<int32_t *>(pinned_host(sizeof(int32_t) * map_entries(r) + sizeof(double) * (am + r.lmax), 1));
    if (!h_vals || !h_map) return fail(CHEBDAV_ENOMEM, "pinned host allocation failed");
    double *h_diag = reinterpret_cast<double *>(h_map + map_entries(r));
    int *h_flag = reinterpret_cast<int *>(h_vals + 2 * am + 2 * r.lmax);

    chebdav_stats S{};
    uint64_t next_col = 0;

    // V_init must be finite
    if (k_init > 0) {
        int *dflag = reinterpret_cast<int *>(L.map);
        CD_HIP(hipMemsetAsync(dflag, 0, sizeof(int), st));
        CD_TRY(check_finite(V_init, k_init, k_init, n, dflag, st));
        CD_HIP(hipMemcpyAsync(h_flag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        if (*h_flag) return fail(CHEBDAV_EINVAL, "V_init holds NaN or Inf");
    }

    // steps 1-3
    const double upperb = r.upperb, lowb = r.lowb;
    double low_nwb = r.low_nwb0;
    {
        const int take = std::min(kb, k_init);
        if (take) CD_TRY((copy_block<double, double>(V_init, k_init, L.Vtmp, kb, take, n, st, g->dinv)));
        if (take < kb) {
            CD_TRY(philox_fill(L.Vtmp + take, n, kb - take, kb, r.seed, next_col, st, g->dinv));
            next_col += kb - take;
            S.n_random += kb - take;
        }
    }
    // Basis bookkeeping.  The active block V(:, kc+1 : ksub) of the algorithm is
    // B Q(:, 1:kact), with B = Va[cur](:, 1:kr) (orthonormal) and the small kr x
    // kact matrix Q[qc]; W[cur](:, 1:kr) = A B.  The columns of B and of the locked
    // vectors Vl(:, kcb+1 : kc) = B Q_locked span the same space as [Vl(:, kcb+1 :
    // kc), B Q], so V(:, 1:ksub) spans [Vl(:, 1:kcb), B], an orthonormal set of
    // kcb + kr = kc + kact = ksub columns.  The tall products B Q and (A B) Q are
    // formed only for the kb leading Ritz pairs (residuals, locking, next block)
    // and, as the rotation of step 11, when a restart drops columns or B is full.
    int ki = kb, kc = 0, kact = 0, kr = 0, kcb = 0, cur = 0, qc = 0;
    std::vector<double> locked;  // eigenvalues in locking order (column order of Vl)
    bool use_f64_filter = r.fdt == CHEBDAV_F64;
    EventPair evp;
    if (r.timing) {
        CD_HIP(hipEventCreate(&evp.b));
        CD_HIP(hipEventCreate(&evp.e));
    }
    CD_TRY(fill_f64(L.ones, am, 1.0, st));
    const int64_t tblk = (int64_t)(align_up((size_t)n * kb * sizeof(double), 256) / sizeof(double));
    double *T0 = static_cast<double *>(L.filt), *T1 = T0 + tblk;  // filter scratch, free between filters
    // rotation: B <- B Q(:, 1:keep), A B <- (A B) Q(:, 1:keep), Q <- I
    auto compress = [&](int keep) -> chebdav_status {
        Seg2 vs, wsg;
        vs.X1 = L.Va[cur];
        vs.ld1 = am;
        vs.p1 = kr;
        wsg.X1 = L.W[cur];
        wsg.ld1 = am;
        wsg.p1 = kr;
        CD_TRY(update(vs, L.Q[qc], am, 1.0, 0.0, L.Va[1 - cur], am, keep, n, st));
        CD_TRY(update(wsg, L.Q[qc], am, 1.0, 0.0, L.W[1 - cur], am, keep, n, st));
        cur = 1 - cur;
        CD_TRY(h_set_diag(L.Q[qc], am, L.ones, keep, st));
        kr = keep;
        kcb = kc;
        return CHEBDAV_OK;
    };
    chebdav_status result = CHEBDAV_ENOCONV;
    // Exit certificate (reading of step 12 with Table 1's extra SpMM): the kout
    // smallest locked pairs, ascending, are written to evals / evecs and their
    // fresh residuals ||A v - lambda v||_2 (one new sparse product) read back into
    // fres; ord[t] is the locked-order column of the t-th smallest.
    std::vector<int> ord;
    std::vector<double> fres;
    bool written = false;
    auto certify = [&](int kout) -> chebdav_status {
        CD_HIP(hipStreamSynchronize(st));  // earlier uploads from the pinned maps have completed
        ord.resize(kc);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return locked[x] < locked[y]; });
        int32_t *m_cert = h_map + map_cert(r);
        for (int t = 0; t < kout; ++t) {
            m_cert[t] = ord[t];
            h_diag[t] = locked[ord[t]];
        }
        CD_HIP(hipMemcpyAsync(L.map + map_cert(r), m_cert, sizeof(int32_t) * kout, hipMemcpyHostToDevice, st));
        CD_HIP(hipMemcpyAsync(L.ev, h_diag, sizeof(double) * kout, hipMemcpyHostToDevice, st));
        CD_TRY(gather_cols(L.Vl, r.lmax, evecs, r.k_want, L.map + map_cert(r), kout, n, st));
        CD_TRY((copy_block<double, double>(L.ev, 1, evals, 1, 1, kout, st)));
        double *tmp = L.W[1 - cur];  // free outside a rotation
        for (int c0 = 0; c0 < kout; c0 += am) {
            const int w = std::min(am, kout - c0);
            CD_TRY((launch_cheb_step<double, double>(g, -1.0, 1.0, 0.0, evecs + c0, r.k_want, nullptr, 0, tmp,
                                                     am, w, st)));
            CD_TRY(colnorms(tmp, am, evecs + c0, r.k_want, L.ev + c0, w, n, L.res + c0, L.part, st));
        }
        S.n_spmm_other += 1;
        CD_HIP(hipMemcpyAsync(h_vals, L.res, sizeof(double) * kout, hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        fres.assign(h_vals, h_vals + kout);
        written = true;
        return CHEBDAV_OK;
    };
    int it = 0, cert_rounds = 0;
    bool cert_failed = false;
    double f32_best = INFINITY;  // smallest open residual seen while filtering in FP32
    double f32_best_max = INFINITY;  // smallest value of the largest wanted open residual in FP32
    int f32_stall = 0;           // FP32 iterations in a row without progress
    std::vector<double> D(am), res(kb);
    while (it < r.itmax) {
        ++it;
        chebdav_iter_record rec{};
        rec.iteration = it;
        rec.low_nwb = low_nwb;
        rec.filter_f32 = !use_f64_filter;
        double *Xnew = L.Va[cur] + kr;
        // step 5: filter
        const chebdav_dtype fdt = use_f64_filter ? CHEBDAV_F64 : CHEBDAV_F32;
        CD_TRY(run_filter(g, L.Vtmp, kb, Xnew, am, kb, r.m, low_nwb, upperb, lowb, fdt, L.filt, L.filt_b,
                          st, evp.b, evp.e, true));
        S.n_spmm_filter += r.m;
        if (fdt == CHEBDAV_F32) S.n_spmm_filter_f32 += r.m;
        // step 6: orthonormalize against V(:, 1:ksub), spanned by [Vl(:, 1:kcb), B]
        Seg2 V;
        V.X1 = L.Vl;
        V.ld1 = r.lmax;
        V.p1 = kcb;
        V.X2 = L.Va[cur];
        V.ld2 = am;
        V.p2 = kr;
        int nrep = 0;
        CD_TRY(orthonormalize(V, Xnew, am, kb, n, r.seed, &next_col, &nrep, L.orthw, L.orth_b, st, r.orth));
        S.n_replaced += nrep;
        S.n_random += nrep;
        if (r.timing) {
            float ms = 0.f;
            CD_HIP(hipEventElapsedTime(&ms, evp.b, evp.e));  // orthonormalize synchronized the stream
            S.t_filter_ms += ms;
            S.n_filter_launches += r.m;
        }
        // step 7: W(:, kr+1 : kr+kb) = A V_new
        CD_TRY((launch_cheb_step<double, double>(g, -1.0, 1.0, 0.0, Xnew, am, nullptr, 0, L.W[cur] + kr, am,
                                                 kb, st)));
        S.n_spmm_other += 1;
        // step 8: H(1:kact+kb, new) = [B Q, V_new]^T A V_new, symmetrized
        {
            Seg2 bs;
            bs.X1 = L.Va[cur];
            bs.ld1 = am;
            bs.p1 = kr + kb;
            CD_TRY(gram(bs, L.W[cur] + kr, am, kb, n, L.C, kb, L.part, st));
            CD_TRY(proj_cols(L.Q[qc], am, L.C, kr, kact, kb, L.C2, st));
            CD_TRY(h_insert(L.H, am, L.C2, kact + kb, kb, st));
        }
        // step 9: H Y = Y D, ascending; Q <- [[Q, 0], [0, I]] Y
        CD_TRY(small_eig(L.H, am, kact + kb, L.D, L.Y, am, L.eigw, L.eig_b, st));
        CD_TRY(extend_basis(L.Q[qc], am, L.Y, am, kr, kact, kb, kact + kb, L.Q[1 - qc], am, st));
        qc = 1 - qc;
        kr += kb;
        kact += kb;
        // steps 10-11: inner restart, with the rotation
        bool rotated = false;
        if (kact + kb > am) {
            kact = r.k_ri;
            CD_TRY(compress(kact));
            rotated = true;
            S.n_inner_restarts += 1;
        }
        rec.kc = kc;
        rec.kact = kact;
        rec.ksub = kc + kact;
        rec.inner_restart = rotated;
        // step 12: residuals of the first kb active pairs, from PV = B Q(:, 1:nres)
        // and PW = (A B) Q(:, 1:nres) (the rotated blocks themselves after a restart)
        const int nres = std::min(kb, kact);
        const double *PV = L.Va[cur], *PW = L.W[cur];
        int64_t ldp = am;
        if (!rotated) {
            Seg2 vs, wsg;
            vs.X1 = L.Va[cur];
            vs.ld1 = am;
            vs.p1 = kr;
            wsg.X1 = L.W[cur];
            wsg.ld1 = am;
            wsg.p1 = kr;
            CD_TRY(update(vs, L.Q[qc], am, 1.0, 0.0, T0, kb, nres, n, st));
            CD_TRY(update(wsg, L.Q[qc], am, 1.0, 0.0, T1, kb, nres, n, st));
            PV = T0;
            PW = T1;
            ldp = kb;
        }
        CD_TRY(colnorms(PW, ldp, PV, ldp, L.D, nres, n, L.res, L.part, st));
        CD_HIP(hipMemcpyAsync(h_vals, L.D, sizeof(double) * (am + nres), hipMemcpyDeviceToHost, st));
        CD_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < kact; ++i) D[i] = h_vals[i];
        for (int i = 0; i < nres; ++i) res[i] = h_vals[am + i];
        std::vector<int> conv, rest;
        for (int i = 0; i < kact; ++i) {
            if (i < nres && res[i] <= r.tol)
                conv.push_back(i);
            else
                rest.push_back(i);
        }
        const int ec = (int)conv.size();
        double min_open_res = INFINITY;
        rec.min_residual = INFINITY;
        rec.max_residual = 0.0;
        double max_open_res = 0.0;  // largest open residual among the wanted pairs
        const int n_wanted = std::min(nres, r.k_want - kc);
        // Ritz value of the last wanted pair, when the kb evaluated pairs hold every
        // wanted pair not yet locked (else NaN)
        const double theta_last = (r.k_want - kc <= nres && n_wanted > 0) ? D[n_wanted - 1] : NAN;
        for (int i = 0; i < nres; ++i) {
            if (!(res[i] <= r.tol)) min_open_res = std::min(min_open_res, res[i]);
            if (!(res[i] <= r.tol) && i < n_wanted) max_open_res = std::max(max_open_res, res[i]);
            rec.min_residual = std::min(rec.min_residual, res[i]);
            rec.max_residual = std::max(rec.max_residual, res[i]);
        }
        rec.n_locked = ec;
        // host decisions first (steps 12-16), then one upload of the maps and the new diagonal
        bool done = kc + ec >= r.k_want;
        int kact_next = kact - ec;
        bool outer = false;
        if (!done && kc + ec + kact_next + kb > r.dim_max) {
            kact_next = r.ro_size(kc + ec);
            outer = true;
        }
        int32_t *m_conv = h_map, *m_rest = h_map + am;
        for (int t = 0; t < ec; ++t) m_conv[t] = conv[t];
        for (int t = 0; t < (int)rest.size(); ++t) m_rest[t] = rest[t];
        std::vector<double> Dact(rest.size());
        for (size_t t = 0; t < rest.size(); ++t) Dact[t] = D[rest[t]];
        if (!done)
            for (int t = 0; t < kact_next; ++t) h_diag[t] = Dact[t];
        const size_t up_bytes = reinterpret_cast<char *>(h_diag + (done ? 0 : kact_next)) - reinterpret_cast<char *>(h_map);
        if (ec || !done) CD_HIP(hipMemcpyAsync(L.map, h_map, up_bytes, hipMemcpyHostToDevice, st));
        if (ec) {
            // lock: append the converged Ritz vectors to Vl
            CD_TRY(gather_cols(PV, ldp, L.Vl + kc, r.lmax, L.map, ec, n, st));
            for (int t = 0; t < ec; ++t) locked.push_back(D[conv[t]]);
            kc += ec;
            // steps 12/14: the non-converged columns of Q move to the front
            if (!rest.empty()) CD_TRY(gather_cols(L.Q[qc], am, L.Q[qc], am, L.map + am, (int)rest.size(), kr, st));
            kact -= ec;
        }
        // step 13, with the exit certificate: pairs whose fresh residual fails are
        // un-locked (the kb smallest first) together with the locked pairs above
        // rank k_want - 1 that would otherwise end the loop again at once; they
        // lead the next block to filter.
        int nu = 0;
        if (done) {
            CD_TRY(certify(r.k_want));
            std::vector<int> bad;
            for (int t = 0; t < r.k_want; ++t)
                if (!(fres[t] <= r.certify_tol)) bad.push_back(t);
            if (bad.empty()) {
                result = CHEBDAV_OK;
            } else if (cert_rounds < r.refine_sweeps) {
                ++cert_rounds;
                if ((int)bad.size() > kb) bad.resize(kb);
                std::vector<char> out(kc, 0);
                for (int t : bad) out[t] = 1;
                for (int t = kc - 1; t >= 0 && kc - (int)std::count(out.begin(), out.end(), 1) >= r.k_want; --t) out[t] = 1;
                std::vector<int> unl, keep;  // locked-order columns
                for (int t = 0; t < kc; ++t) (out[t] ? unl : keep).push_back(ord[t]);
                std::sort(keep.begin(), keep.end());
                nu = (int)unl.size();
                const int kc_new = kc - nu;
                // B must hold no locked vector before the locked set shrinks: rotate
                // it to the retained active pairs, with step 16's size for kc_new
                kact_next = kact;
                if (kc_new + kact + kb > r.dim_max) {
                    kact_next = r.ro_size(kc_new);
                    outer = true;
                }
                int32_t *m_unl = h_map + map_unl(r), *m_keep = h_map + map_keep(r);
                for (int t = 0; t < nu; ++t) m_unl[t] = unl[t];
                for (int t = 0; t < kc_new; ++t) m_keep[t] = keep[t];
                for (int t = 0; t < kact_next; ++t) h_diag[t] = Dact[t];
                const size_t ub = reinterpret_cast<char *>(h_diag + kact_next) - reinterpret_cast<char *>(h_map);
                CD_HIP(hipMemcpyAsync(L.map, h_map, ub, hipMemcpyHostToDevice, st));  // certify synchronized
                kact = kact_next;
                CD_TRY(compress(kact));
                CD_TRY(gather_cols(L.Vl, r.lmax, L.Vtmp, kb, L.map + map_unl(r), nu, n, st, g->dinv));
                if (kc_new) CD_TRY(gather_cols(L.Vl, r.lmax, L.Vl, r.lmax, L.map + map_keep(r), kc_new, n, st));
                std::vector<double> lk(kc_new);
                for (int t = 0; t < kc_new; ++t) lk[t] = locked[keep[t]];
                locked.swap(lk);
                kc = kcb = kc_new;
                S.used_fallback = 1;
                S.n_unlocked += nu;
                use_f64_filter = true;
                done = false;
                written = false;  // the next exit writes the outputs again
            } else {
                cert_failed = true;
            }
        }
        rec.n_unlocked = nu;
        if (done) {
            rec.outer_restart = 0;
            if (r.log_cb) r.log_cb(&rec, r.log_user);
            break;
        }
        // step 16: outer restart (ksub = kc + kact); B also rotated when it is full
        if (nu == 0) {
            if (outer) {
                kact = kact_next;
                CD_TRY(compress(kact));
            } else if (kr + kb > am) {
                CD_TRY(compress(kact));
            }
        }
        if (outer) S.n_outer_restarts += 1;
        rec.outer_restart = outer;
        // step 15: H = diag of the retained non-converged Ritz values
        if (kact) CD_TRY(h_set_diag(L.H, am, L.hd, kact, st));
        // step 17: next block = [un-locked pairs, unused V_init columns, leading Ritz vectors, random]
        {
            const int n_init = std::max(0, std::min(std::min(ec, k_init - ki), kb - nu));
            const int n_ritz = std::min(std::min(kb - ec, kact), kb - nu - n_init);
            const int pad = kb - nu - n_init - n_ritz;
            double *vt = L.Vtmp + nu;
            if (n_init) CD_TRY((copy_block<double, double>(V_init + ki, k_init, vt, kb, n_init, n, st, g->dinv)));
            if (n_ritz) {
                // the leading non-converged pairs are all among the first nres columns of PV
                if (ec)
                    CD_TRY(gather_cols(PV, ldp, vt + n_init, kb, L.map + am, n_ritz, n, st, g->dinv));
                else
                    CD_TRY((copy_block<double, double>(PV, ldp, vt + n_init, kb, n_ritz, n, st, g->dinv)));
            }
            if (pad) {
                CD_TRY(philox_fill(vt + n_init + n_ritz, n, pad, kb, r.seed, next_col, st, g->dinv));
                next_col += pad;
                S.n_random += pad;
            }
            ki += n_init;
        }
        // step 18
        if (kact) {
            const double med = median_of(std::vector<double>(Dact.begin(), Dact.begin() + kact));
            if (lowb < med && med < upperb) low_nwb = med;
        }
        // mixed precision: when to filter in FP64 from now on.
        // (a) When the evaluated block holds every wanted pair still open and their
        //     Ritz pairs are accurate enough to predict the filter's effect (the
        //     largest wanted residual is at most a tenth of the distance from the
        //     last wanted Ritz value theta up to the next cut, so the eigenvalue it
        //     approximates is that far below the cut too): per FP64 iteration the
        //     filter of Alg. 3 divides that pair's residual by about
        //     |C_m((theta - c) / e)| (unwanted components stay below 1 in size),
        //     while one more FP32 iteration does the same but stops at the FP32
        //     floor f32_switch_tol.  Switch as soon as one more FP32 iteration would
        //     not save an FP64 iteration.
        // (b) Otherwise once the smallest open residual reaches that floor.
        // (c) Either way once FP32 filtering stops making progress on the wanted
        //     block: two iterations in a row that neither locked a pair nor halved
        //     the smallest open residual nor the largest wanted open residual.
        if (!use_f64_filter) {
            if (ec > 0 || min_open_res < 0.5 * f32_best || max_open_res < 0.5 * f32_best_max) {
                f32_stall = 0;
            } else {
                ++f32_stall;
            }
            f32_best = std::min(f32_best, min_open_res);
            f32_best_max = std::min(f32_best_max, max_open_res);
            bool to_f64;
            if (theta_last < low_nwb && max_open_res <= 0.1 * (low_nwb - theta_last)) {
                const double c = 0.5 * (low_nwb + upperb), e = 0.5 * (upperb - low_nwb);
                const double gain = std::cosh(r.m * std::acosh((c - theta_last) / e));  // |C_m| > 1
                auto fp64_its = [&](double res0) {
                    if (res0 <= r.tol) return 0.0;
                    return std::max(1.0, std::ceil(std::log(res0 / r.tol) / std::log(gain)));
                };
                to_f64 = fp64_its(max_open_res) <= fp64_its(std::max(max_open_res / gain, r.f32_switch_tol));
            } else {
                to_f64 = min_open_res < r.f32_switch_tol;
            }
            if (to_f64 || f32_stall >= 2) use_f64_filter = true;
        }
        if (r.log_cb) r.log_cb(&rec, r.log_user);
    }
    S.iterations = it;
    // outputs: the certificate of the loop's exit, or (itmax) of the locked pairs found
    if (!written) {
        const int kout = std::min(kc, r.k_want);
        if (kout > 0)
            CD_TRY(certify(kout));
        else
            fres.clear();
    }
    int n_cert = 0;
    double mr = fres.empty() ? NAN : 0.0;
    for (double f : fres) {
        mr = std::max(mr, f);
        n_cert += f <= r.certify_tol;
    }
    S.max_residual = mr;
    S.converged = n_cert;
    CD_HIP(hipStreamSynchronize(st));
    S.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = S;
    if (result != CHEBDAV_OK) {
        if (cert_failed)
            return fail(CHEBDAV_ENOCONV, "exit certificate failed for %d of %d pairs after %d refinement rounds",
                        r.k_want - n_cert, r.k_want, cert_rounds);
        return fail(result, "itmax reached with %d of %d pairs certified", n_cert, r.k_want);
    }
    return CHEBDAV_OK;
}

}  // namespace chebdav
