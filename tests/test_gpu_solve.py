"""GPU parity for the full solver (Alg. 2) against the oracle: eigenvalues
|d lambda| <= 1e-10, fresh residuals <= 1e-8, largest principal angle <= 1e-6,
iteration counts within +-2; closed-form spectra; error paths."""

import math

import numpy as np
import pytest

import synth
from conftest import sin_max_angle

pytestmark = pytest.mark.gpu


def _gpu_solve(cd, edges, n, V_init=None, **kw):
    import torch
    g = cd.build_laplacian(edges, n)
    p = cd.make_params(**kw)
    vi = None if V_init is None else torch.from_numpy(np.ascontiguousarray(V_init)).cuda()
    r = cd.solve(g, p, V_init=vi)
    return g, r.evals.cpu().numpy(), r.evecs.cpu().numpy(), r.stats


def _fresh_residuals(o, evals, evecs):
    R = o.apply_laplacian(o_csr_cache[0], np.asfortranarray(evecs)) - evecs * evals
    return np.sqrt((R * R).sum(0))


o_csr_cache = [None]


def _parity(cd, oracle_mod, edges, n, k, kb, m, seed=1, it_slack=2, gpu_kw=None, **kw):
    o = oracle_mod.build_csr(edges, n)
    o_csr_cache[0] = o
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=k, kb=kb, m=m, seed=seed, **kw))
    _, ev, V, st = _gpu_solve(cd, edges, n, k_want=k, kb=kb, m=m, seed=seed, **kw, **(gpu_kw or {}))
    res = _fresh_residuals(oracle_mod, ev, V)
    print("iters gpu %d oracle %d; max res %.3g; max dlam %.3g" %
          (st["iterations"], ref.iterations, res.max(), np.abs(ev - ref.evals).max()))
    assert st["converged"] >= k
    assert res.max() <= 1e-8
    assert st["max_residual"] <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= 1e-12
    assert abs(st["iterations"] - ref.iterations) <= it_slack
    return ev, V, st, ref


def test_sbm5k_parity(cd, oracle_mod, dev):
    e, n, _ = synth.make_config_graph("sbm5k")
    ev, V, st, ref = _parity(cd, oracle_mod, e, n, 4, 4, 11)
    assert sin_max_angle(ref.evecs, V) <= 1e-6


def test_sbm20k_k16_parity(cd, oracle_mod, dev):
    e, _ = synth.sbm(20_000, 16, d_in=20, d_out=4, uneven=True, seed=3)
    ev, V, st, ref = _parity(cd, oracle_mod, e, 20_000, 16, 8, 15, seed=7)
    assert sin_max_angle(ref.evecs, V) <= 1e-6


@pytest.mark.parametrize("k,kb,m", [(12, 7, 9), (11, 5, 11), (12, 12, 7), (5, 1, 15), (13, 3, 13)])
def test_block_sizes_parity(cd, oracle_mod, dev, k, kb, m):
    """Block sizes off the powers of two (kb = 3, 5, 7: padded sparse-step columns and
    partial MFMA tiles), single-vector blocks (kb = 1), k not a multiple of kb and kb = k,
    on a 6000-node SBM whose 12 planted blocks put a gap of 0.43 after the 12th
    eigenvalue (inner restarts fire in four of the five cases).  The subspace angle is
    checked for k = 12, the only case with a gap above 0.01 after the k-th eigenvalue."""
    e, _ = synth.sbm(6000, 12, d_in=18, d_out=3, uneven=True, seed=11)
    print("case block sizes k=%d kb=%d m=%d" % (k, kb, m), flush=True)
    ev, V, st, ref = _parity(cd, oracle_mod, e, 6000, k, kb, m, seed=3, it_slack=3 if kb == 1 else 2)
    if k == 12:
        assert sin_max_angle(ref.evecs, V) <= 1e-6


def test_dense_eigh_small(cd, oracle_mod, dev):
    n = 1500
    e, _ = synth.sbm(n, 6, d_in=12, d_out=2, uneven=True, seed=4)
    o = oracle_mod.build_csr(e, n)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(o))
    _, ev, V, st = _gpu_solve(cd, e, n, k_want=6, kb=3, m=11, seed=2)
    assert np.abs(ev - lam[:6]).max() <= 1e-10
    assert sin_max_angle(Q[:, :6], V) <= 1e-6


@pytest.mark.parametrize("name", ["cycle", "path", "complete", "bipartite", "hypercube", "components"])
def test_closed_form_spectra(cd, oracle_mod, dev, name):
    kw = dict(kb=4, m=11, seed=3)
    if name == "cycle":
        n = 200
        e, k = synth.cycle_graph(n), 5
        want = np.sort([1 - math.cos(2 * math.pi * j / n) for j in (0, 1, 1, 2, 2)])
    elif name == "path":
        n = 120
        e, k = synth.path_graph(n), 6
        kw["kb"], kw["m"] = 3, 15
        want = np.array([1 - math.cos(math.pi * j / (n - 1)) for j in range(6)])
    elif name == "complete":
        n = 60
        e, k = synth.complete_graph(n), 4
        want = np.array([0.0] + [n / (n - 1)] * 3)
    elif name == "bipartite":
        n = 50
        e, k = synth.complete_bipartite_graph(20, 30), 3
        kw.update(kb=3, act_max=15, dim_max=21)
        want = np.array([0.0, 1.0, 1.0])
    elif name == "hypercube":
        d = 7
        n = 1 << d
        e, k = synth.hypercube_graph(d), 1 + d
        want = np.array([0.0] + [2.0 / d] * d)
    else:
        parts = [(synth.cycle_graph(50), 50), (synth.path_graph(40), 40), (synth.complete_graph(30), 30),
                 (np.zeros((0, 2), np.int64), 2)]
        e, n = synth.disjoint_union(parts)
        k = 3
        want = np.zeros(3)
    print("case closed form %s" % name, flush=True)
    g, ev, V, st = _gpu_solve(cd, e, n, k_want=k, **kw)
    o = oracle_mod.build_csr(e, n)
    o_csr_cache[0] = o
    assert np.abs(ev - want).max() <= 1e-10
    assert _fresh_residuals(oracle_mod, ev, V).max() <= 1e-8
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= 1e-12


def test_warm_start_exact(cd, oracle_mod, dev):
    n = 1500
    e, _ = synth.sbm(n, 4, p_in=0.05, p_out=0.003, seed=9)
    o = oracle_mod.build_csr(e, n)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(o))
    _, ev, V, st = _gpu_solve(cd, e, n, V_init=Q[:, :8], k_want=4, kb=4, m=11, seed=1)
    assert st["iterations"] == 1 and st["n_random"] == 0
    assert np.abs(ev - lam[:4]).max() <= 1e-12


def test_itmax_and_errors(cd, dev):
    import torch
    n = 2000
    e, _ = synth.sbm(n, 8, d_in=10, d_out=3, uneven=True, seed=2)
    g = cd.build_laplacian(e, n)
    r = cd.solve(g, cd.make_params(k_want=8, kb=4, m=11, itmax=1), allow_noconv=True)
    assert r.status == cd.ENOCONV and r.stats["iterations"] == 1 and r.stats["converged"] < 8
    bad = torch.full((n, 4), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(cd.ChebdavError) as ei:
        cd.solve(g, cd.make_params(k_want=4, kb=4, m=11), V_init=bad)
    assert ei.value.status == cd.EINVAL
    with pytest.raises(cd.ChebdavError) as ei:
        cd.solve(g, cd.make_params(k_want=100, kb=4, m=5, dim_max=60))
    assert ei.value.status == cd.EINVAL
    with pytest.raises(cd.ChebdavError) as ei:
        cd.solve(g, cd.make_params(k_want=4, kb=4, m=0))
    assert ei.value.status == cd.EINVAL


def test_deterministic(cd, dev):
    e, n, _ = synth.make_config_graph("sbm5k")
    _, ev1, V1, s1 = _gpu_solve(cd, e, n, k_want=4, kb=4, m=11, seed=5)
    _, ev2, V2, s2 = _gpu_solve(cd, e, n, k_want=4, kb=4, m=11, seed=5)
    assert np.array_equal(ev1, ev2) and np.array_equal(V1, V2)
    assert s1["iterations"] == s2["iterations"]


def test_f32_form_sbm20k(cd, oracle_mod, dev):
    e, _ = synth.sbm(20_000, 16, d_in=20, d_out=4, uneven=True, seed=3)
    n = 20_000
    o = oracle_mod.build_csr(e, n)
    o_csr_cache[0] = o
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=16, kb=8, m=15, seed=7))
    _, ev, V, st = _gpu_solve(cd, e, n, k_want=16, kb=8, m=15, seed=7, filter_dtype=cd.F32)
    res = _fresh_residuals(oracle_mod, ev, V)
    print("f32 form: iters %d (f32 steps %d of %d), max res %.3g, max dlam %.3g" %
          (st["iterations"], st["n_spmm_filter_f32"], st["n_spmm_filter"], res.max(),
           np.abs(ev - ref.evals).max()))
    assert res.max() <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    assert st["n_spmm_filter_f32"] > 0


_full = {}


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_sbm200k_full_size_parity(cd, oracle_mod, dev, form):
    """The 200k-node, 32-block workload at full size (k = kb = 32, m = 15),
    in the configuration the benchmark times, against the full oracle solve."""
    e, n, cfg = synth.make_config_graph("sbm200k")
    if "ref" not in _full:
        o = oracle_mod.build_csr(e, n)
        _full["o"] = o
        _full["ref"] = oracle_mod.bchdav(o, oracle_mod.Params(k_want=32, kb=32, m=15, seed=1))
    o, ref = _full["o"], _full["ref"]
    o_csr_cache[0] = o
    print("case sbm200k full solve %s" % form, flush=True)
    _, ev, V, st = _gpu_solve(cd, e, n, k_want=32, kb=32, m=15, seed=1,
                              filter_dtype=cd.F64 if form == "f64" else cd.F32)
    res = _fresh_residuals(oracle_mod, ev, V)
    print("sbm200k %s: iters gpu %d oracle %d; max res %.3g; max dlam %.3g; angle %.3g" %
          (form, st["iterations"], ref.iterations, res.max(), np.abs(ev - ref.evals).max(),
           sin_max_angle(ref.evecs, V)))
    assert res.max() <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    assert np.linalg.norm(V.T @ V - np.eye(32), 2) <= 1e-12
    if form == "f64":
        assert abs(st["iterations"] - ref.iterations) <= 2


def test_streaming_warm_start(cd, oracle_mod, dev):
    """Warm start from the eigenvectors of a slightly different graph (the
    streaming-graph use of V_init, Alg. 2 steps 2 and 17): after 0.5% of the
    edges are rewired, the previous eigenvectors, passed as V_init, are filtered
    progressively and reach the new eigenpairs with fewer iterations than a
    random start.  The oracle runs the same sequence on its own: it solves the
    old graph, then the new one from its own previous eigenvectors; the GPU's
    warm solve must match it to the solve bar, iterations within +-2."""
    import torch
    e, n, cfg = synth.make_config_graph("sbm200k")
    g0 = cd.build_laplacian(e, n)
    p = cd.make_params(k_want=32, kb=32, m=15, seed=1)
    prev = cd.solve(g0, p)
    rng = np.random.default_rng(5)
    keep = rng.random(len(e)) >= 0.005
    new = rng.integers(0, n, size=(int((~keep).sum()), 2))
    e2 = np.concatenate([e[keep], new]).astype(np.int64)
    g1 = cd.build_laplacian(e2, n)
    rnd = cd.solve(g1, p)
    warm = cd.solve(g1, p, V_init=prev.evecs.contiguous())
    o0 = oracle_mod.build_csr(e, n)
    o = oracle_mod.build_csr(e2, n)
    o_prev = oracle_mod.bchdav(o0, oracle_mod.Params(k_want=32, kb=32, m=15, seed=1))
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=32, kb=32, m=15, seed=1), V_init=o_prev.evecs)
    V, ev = warm.evecs.cpu().numpy(), warm.evals.cpu().numpy()
    R = oracle_mod.apply_laplacian(o, np.asfortranarray(V)) - V * ev
    print("streaming: random start %d iterations, previous-eigenvector start %d iterations (oracle %d)"
          % (rnd.stats["iterations"], warm.stats["iterations"], ref.iterations))
    assert np.sqrt((R * R).sum(0)).max() <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    assert abs(warm.stats["iterations"] - ref.iterations) <= 2
    assert np.abs(ev - rnd.evals.cpu().numpy()).max() <= 1e-10
    assert warm.stats["iterations"] < rnd.stats["iterations"]


def test_concurrent_solves_two_threads(cd, dev):
    """Two host threads solve at the same time, each on its own stream with its
    own workspace and the graph handle shared: the library keeps no mutable
    global state (per-thread pinned scratch and error text), so each result
    equals the sequential solve bit for bit."""
    import threading
    import torch
    n = 20_000
    e, _ = synth.sbm(n, 8, d_in=20, d_out=4, uneven=True, seed=11)
    g = cd.build_laplacian(e, n)
    params = [cd.make_params(k_want=8, kb=8, m=11, seed=s) for s in (1, 2)]
    ref = []
    for p in params:
        r = cd.solve(g, p)
        ref.append((r.evals.cpu().numpy(), r.evecs.cpu().numpy()))
    out, errs = [None, None], []

    def run(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                r = cd.solve(g, params[i], stream=s)
                s.synchronize()
                out[i] = (r.evals.cpu().numpy(), r.evecs.cpu().numpy())
        except Exception as ex:  # reported below
            errs.append(ex)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for i in range(2):
        assert np.array_equal(out[i][0], ref[i][0])
        assert np.array_equal(out[i][1], ref[i][1])


def _trajectory(rows):
    return [(r["kc"], r["kact"], r["ksub"], bool(r["inner_restart"]), bool(r["outer_restart"])) for r in rows]


@pytest.mark.parametrize("case", ["sbm5k_16blocks", "sbm20k_64blocks"])
def test_outer_restart_parity(cd, oracle_mod, dev, case):
    """Alg. 2 step 16: k_want well above 2 kb + 1 makes the search space reach
    dim_max, so the outer restart cuts it to dim_max - 2 kb - kc columns.  The
    GPU solve matches the oracle's to the solve bar, and its per-iteration
    trajectory (kc, kact, ksub and the restarts, from the iteration log) equals
    the oracle's up to and including the first outer restart."""
    if case == "sbm5k_16blocks":
        n, B, k, kb, m, kw, seed = 5000, 16, 16, 4, 15, dict(act_max=20, dim_max=25), 1
    else:
        n, B, k, kb, m, kw, seed = 20_000, 64, 64, 16, 15, {}, 3
    e, _ = synth.sbm(n, B, d_in=20, d_out=4, uneven=True, seed=seed)
    log = []
    print("case outer restart %s" % case, flush=True)
    ev, V, st, ref = _parity(cd, oracle_mod, e, n, k, kb, m, seed=1, gpu_kw=dict(log=log), **kw)
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    first = next(i for i, h in enumerate(ref.history) if h["outer_restart"])
    assert len(log) == st["iterations"] and st["n_outer_restarts"] >= 1
    assert _trajectory(log[:first + 1]) == _trajectory(ref.history[:first + 1])
    print("outer restarts: gpu %d, oracle %d" % (st["n_outer_restarts"],
                                                 sum(h["outer_restart"] for h in ref.history)))


def test_exit_certificate_unlocks_and_refines(cd, oracle_mod, dev):
    """The exit certificate acts: with certify_tol below tol, every pair passes
    the in-loop test (W - V theta, tol 1e-8) but fails the fresh-product
    certificate, so pairs are un-locked and refined until their fresh residual
    meets certify_tol; the oracle takes the same reading."""
    n = 1500
    e, _ = synth.sbm(n, 4, d_in=16, d_out=3, uneven=True, seed=5)
    o = oracle_mod.build_csr(e, n)
    o_csr_cache[0] = o
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(o))
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1, certify_tol=1e-13))
    _, ev, V, st = _gpu_solve(cd, e, n, k_want=4, kb=4, m=11, seed=1, certify_tol=1e-13)
    res = _fresh_residuals(oracle_mod, ev, V)
    print("certificate: gpu %d iterations, %d un-locked; oracle %d iterations, %d un-locked; max res %.3g"
          % (st["iterations"], st["n_unlocked"], ref.iterations, ref.n_unlocked, res.max()))
    assert st["used_fallback"] == 1 and st["n_unlocked"] >= 1 and st["converged"] == 4
    assert st["max_residual"] <= 1e-13 and res.max() <= 1.1e-13
    assert np.abs(ev - lam[:4]).max() <= 1e-12 and np.abs(ev - ref.evals).max() <= 1e-12
    assert abs(st["iterations"] - ref.iterations) <= 2
    # the plain solve needs no refinement
    _, _, _, st0 = _gpu_solve(cd, e, n, k_want=4, kb=4, m=11, seed=1)
    assert st0["used_fallback"] == 0 and st0["n_unlocked"] == 0 and st0["max_residual"] <= 1e-8


def test_exit_certificate_failure_is_noconv(cd, dev):
    """A certificate no pair can meet ends the solve with ENOCONV after
    refine_sweeps rounds; the pairs are still written and stats.converged counts
    only the certified ones."""
    n = 1500
    e, _ = synth.sbm(n, 4, d_in=16, d_out=3, uneven=True, seed=5)
    g = cd.build_laplacian(e, n)
    r = cd.solve(g, cd.make_params(k_want=4, kb=4, m=11, seed=1, certify_tol=1e-30, refine_sweeps=2),
                 allow_noconv=True)
    assert r.status == cd.ENOCONV
    assert r.stats["converged"] < 4 and r.stats["used_fallback"] == 1
    assert r.stats["n_unlocked"] >= 2 and np.isfinite(r.evals.cpu().numpy()).all()


@pytest.mark.slow
def test_chung_lu_500k_oracle_parity(cd, oracle_mod, dev):
    """A full solve on a Chung-Lu graph from the 8M-node workload's generator at
    500k nodes (hub rows of degree ~800, no planted clusters), k = kb = 32,
    m = 20, against the oracle's full solve.  Eigenvalues are pinned at 1e-10 by
    the residual bound (Kato-Temple).  The graph has no planted clusters: the
    gap after the 32nd eigenvalue is only 2.3e-3 (the oracle's 36 smallest:
    0.234955 then 0.237232), so Davis-Kahan bounds each solution's angle to the
    exact subspace by sqrt(32) 1e-8 / 2.3e-3 = 2.5e-5, and the two solutions'
    largest principal angle by twice that.  The FP32-filter form (its switch to
    FP64 predicted from the Chebyshev rate at the last wanted Ritz value) is held
    to the same bar against the same oracle solve."""
    e, n = synth.chung_lu(500_000, seed=synth.graphs.DEFAULT_SEED + 4)
    print("case chung-lu 500k full solve (n=%d)" % n, flush=True)
    ev, V, st, ref = _parity(cd, oracle_mod, e, n, 32, 32, 20, seed=1)
    ang = sin_max_angle(ref.evecs, V)
    print("chung-lu 500k: largest principal angle %.3g" % ang)
    assert ang <= 1e-4
    print("case chung-lu 500k FP32 form", flush=True)
    _, ev32, V32, st32 = _gpu_solve(cd, e, n, k_want=32, kb=32, m=20, seed=1, filter_dtype=cd.F32)
    res32 = _fresh_residuals(oracle_mod, ev32, V32)
    print("chung-lu 500k FP32 form: %d iterations (FP32 steps %d of %d), max res %.3g, max dlam %.3g"
          % (st32["iterations"], st32["n_spmm_filter_f32"], st32["n_spmm_filter"], res32.max(),
             np.abs(ev32 - ref.evals).max()))
    assert res32.max() <= 1e-8 and st32["converged"] >= 32
    assert np.abs(ev32 - ref.evals).max() <= 1e-10
    assert sin_max_angle(ref.evecs, V32) <= 1e-4
    assert 0 < st32["n_spmm_filter_f32"] < st32["n_spmm_filter"]


def test_f32_form_stall_guard(cd, oracle_mod, dev):
    """FP32 form asked for a residual an FP32-filtered block cannot deliver
    (tol 1e-9; FP32 filtering levels off near 4e-8 here) with a switch level it
    cannot reach either (1e-14): the filter must hand over to FP64 once FP32
    iterations stop making progress (none locks a pair or halves the smallest
    open residual or the largest wanted open residual, twice in a row), and the solve then converges to the oracle's
    eigenpairs at that tolerance."""
    n = 20_000
    e, _ = synth.sbm(n, 16, d_in=20, d_out=4, uneven=True, seed=3)
    o = oracle_mod.build_csr(e, n)
    o_csr_cache[0] = o
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=16, kb=8, m=15, seed=7, tol=1e-9))
    assert ref.status == "ok"
    log = []
    _, ev, V, st = _gpu_solve(cd, e, n, k_want=16, kb=8, m=15, seed=7, tol=1e-9, filter_dtype=cd.F32,
                              f32_switch_tol=1e-14, log=log)
    res = _fresh_residuals(oracle_mod, ev, V)
    flags = [r["filter_f32"] for r in log]
    print("stall guard: %d iterations (oracle %d), FP32 steps %d of %d, filter per iteration %s, max res %.3g"
          % (st["iterations"], ref.iterations, st["n_spmm_filter_f32"], st["n_spmm_filter"],
             "".join("4" if f else "8" for f in flags), res.max()))
    assert st["converged"] == 16 and res.max() <= 1e-9 * 1.01
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    assert 0 < st["n_spmm_filter_f32"] < st["n_spmm_filter"]
    k = flags.index(0)
    assert all(flags[:k]) and not any(flags[k:])
