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


def _parity(cd, oracle_mod, edges, n, k, kb, m, seed=1, it_slack=2, **kw):
    o = oracle_mod.build_csr(edges, n)
    o_csr_cache[0] = o
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=k, kb=kb, m=m, seed=seed, **kw))
    _, ev, V, st = _gpu_solve(cd, edges, n, k_want=k, kb=kb, m=m, seed=seed, **kw)
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
    streaming-graph use of V_init): after 0.5% of the edges are rewired, the
    previous eigenvectors, passed as V_init, are filtered progressively and
    reach the new eigenpairs with fewer iterations than a random start."""
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
    o = oracle_mod.build_csr(e2, n)
    V, ev = warm.evecs.cpu().numpy(), warm.evals.cpu().numpy()
    R = oracle_mod.apply_laplacian(o, np.asfortranarray(V)) - V * ev
    print("streaming: random start %d iterations, previous-eigenvector start %d iterations"
          % (rnd.stats["iterations"], warm.stats["iterations"]))
    assert np.sqrt((R * R).sum(0)).max() <= 1e-8
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
