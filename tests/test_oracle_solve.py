"""Pins for the oracle's block Chebyshev-Davidson solve (Alg. 2): dense
eigendecomposition (LAPACK) for n <= 2000, closed-form normalized-Laplacian
spectra, and the invariants of Eq. 2 (0 <= lambda <= 2, lambda_1 = 0 with
eigenvector proportional to D^{1/2} 1, multiplicity of 0 = number of
components with at least two nodes)."""

import math

import numpy as np
import pytest

import synth


def sin_max_angle(Q1, Q2):
    """sin of the largest principal angle between span(Q2) and span(Q1),
    ||(I - Q1 Q1^T) Q2||_2 (Q1, Q2 orthonormal; span(Q2) of lower or equal dim)."""
    return np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2), 2)


def _solve(o, edges, n, **kw):
    g = o.build_csr(edges, n)
    r = o.bchdav(g, o.Params(**kw))
    return g, r


def _check_common(o, g, r, k, tol=1e-8):
    assert r.converged >= k
    assert r.evals.shape == (k,) and r.evecs.shape == (g.n, k)
    assert (np.diff(r.evals) >= 0).all()
    assert r.max_residual <= tol
    assert np.linalg.norm(r.evecs.T @ r.evecs - np.eye(k), 2) < 1e-12
    assert r.evals.min() > -1e-12 and r.evals.max() < 2 + 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_sbm_against_dense_eigh(oracle_mod, seed):
    n = 2000
    e, _ = synth.sbm(n, 4, p_in=0.04, p_out=0.002, seed=seed)
    g, r = _solve(oracle_mod, e, n, k_want=4, kb=4, m=11, seed=seed)
    _check_common(oracle_mod, g, r, 4)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(g))
    assert np.abs(r.evals - lam[:4]).max() <= 1e-10
    assert lam[4] - lam[3] > 0.1
    assert sin_max_angle(Q[:, :4], r.evecs) <= 1e-6
    # lambda_1 = 0 with eigenvector proportional to D^{1/2} 1 (connected graph)
    v = np.sqrt(g.deg.astype(float))
    v /= np.linalg.norm(v)
    assert abs(r.evals[0]) < 1e-12
    assert sin_max_angle(r.evecs[:, :1], v[:, None]) < 1e-7


def test_sbm_more_vectors_than_block(oracle_mod):
    n = 2000
    e, _ = synth.sbm(n, 12, d_in=15, d_out=2, uneven=True, seed=5)
    g, r = _solve(oracle_mod, e, n, k_want=12, kb=4, m=15, seed=3)
    _check_common(oracle_mod, g, r, 12)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(g))
    assert np.abs(r.evals - lam[:12]).max() <= 1e-10
    assert sin_max_angle(Q[:, :12], r.evecs) <= 1e-6


def test_cycle_closed_form(oracle_mod):
    n = 200
    g, r = _solve(oracle_mod, synth.cycle_graph(n), n, k_want=5, kb=4, m=11, seed=1)
    _check_common(oracle_mod, g, r, 5)
    want = np.sort([1 - math.cos(2 * math.pi * j / n) for j in (0, 1, 1, 2, 2)])
    assert np.abs(r.evals - want).max() <= 1e-10


def test_path_closed_form(oracle_mod):
    n = 120
    g, r = _solve(oracle_mod, synth.path_graph(n), n, k_want=6, kb=3, m=15, seed=2)
    _check_common(oracle_mod, g, r, 6)
    want = np.array([1 - math.cos(math.pi * j / (n - 1)) for j in range(6)])
    assert np.abs(r.evals - want).max() <= 1e-10


def test_complete_graph(oracle_mod):
    n = 60
    g, r = _solve(oracle_mod, synth.complete_graph(n), n, k_want=4, kb=4, m=11, seed=3)
    _check_common(oracle_mod, g, r, 4)
    assert abs(r.evals[0]) < 1e-12
    assert np.abs(r.evals[1:] - n / (n - 1)).max() <= 1e-10


def test_complete_bipartite(oracle_mod):
    p, q = 20, 30
    g, r = _solve(oracle_mod, synth.complete_bipartite_graph(p, q), p + q, k_want=3, kb=3, m=11,
                  seed=4, act_max=15, dim_max=21)
    _check_common(oracle_mod, g, r, 3)
    assert np.abs(r.evals - np.array([0.0, 1.0, 1.0])).max() <= 1e-10


def test_hypercube(oracle_mod):
    d = 7
    n = 1 << d
    g, r = _solve(oracle_mod, synth.hypercube_graph(d), n, k_want=1 + d, kb=4, m=11, seed=5)
    _check_common(oracle_mod, g, r, 1 + d)
    want = np.array([0.0] + [2.0 / d] * d)
    assert np.abs(r.evals - want).max() <= 1e-10


def test_components_and_isolated_nodes(oracle_mod):
    parts = [(synth.cycle_graph(50), 50), (synth.path_graph(40), 40),
             (synth.complete_graph(30), 30), (np.zeros((0, 2), np.int64), 2)]
    e, n = synth.disjoint_union(parts)
    g, r = _solve(oracle_mod, e, n, k_want=3, kb=4, m=11, seed=6)
    _check_common(oracle_mod, g, r, 3)
    assert np.abs(r.evals).max() < 1e-10                  # three components of size >= 2
    # the 0-eigenspace is spanned by D^{1/2} 1 restricted to each component
    B = np.zeros((n, 3))
    off = 0
    for c, (_, sz) in enumerate(parts[:3]):
        B[off:off + sz, c] = np.sqrt(g.deg[off:off + sz])
        off += sz
    B /= np.linalg.norm(B, axis=0)
    assert sin_max_angle(B, r.evecs) < 1e-7
    # the isolated nodes carry eigenvalue 1: asking for 4 includes no 1 (the
    # fourth eigenvalue is the cycle's/path's smallest positive one)
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(g))
    assert np.sum(np.abs(lam - 1.0) < 1e-12) >= 2


def test_warm_start_exact_vectors(oracle_mod):
    n = 1500
    e, _ = synth.sbm(n, 4, p_in=0.05, p_out=0.003, seed=9)
    g = oracle_mod.build_csr(e, n)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(g))
    r = oracle_mod.bchdav(g, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1), V_init=Q[:, :8])
    assert r.iterations == 1 and r.n_random == 0
    assert np.abs(r.evals - lam[:4]).max() <= 1e-12


def test_itmax_partial(oracle_mod):
    n = 2000
    e, _ = synth.sbm(n, 8, d_in=10, d_out=3, uneven=True, seed=2)
    g = oracle_mod.build_csr(e, n)
    r = oracle_mod.bchdav(g, oracle_mod.Params(k_want=8, kb=4, m=11, itmax=1, seed=0))
    assert r.iterations == 1 and r.converged < 8


def test_parameter_defaults(oracle_mod):
    p = oracle_mod.resolve_params(oracle_mod.Params(k_want=64, kb=64, m=20), 2_000_000)
    assert (p.act_max, p.dim_max, p.k_ri) == (320, 448, 160)
    p = oracle_mod.resolve_params(oracle_mod.Params(k_want=32, kb=32, m=15), 200_000)
    assert (p.act_max, p.dim_max, p.k_ri) == (160, 224, 80)
    p = oracle_mod.resolve_params(oracle_mod.Params(k_want=4, kb=4, m=11), 5000)
    assert (p.act_max, p.dim_max, p.k_ri) == (30, 38, 18)
    assert p.low_nwb0 == pytest.approx(2 * 4 / 5000)
    with pytest.raises(ValueError):
        oracle_mod.resolve_params(oracle_mod.Params(k_want=100, kb=4, m=5, dim_max=60), 5000)


@pytest.mark.parametrize("k_ro", [0, 5])
def test_outer_restart_against_dense(oracle_mod, k_ro):
    """Alg. 2 step 16 fires (k_want = 12 > 2 kb + 1 with a small dim_max): the
    search space is cut to dim_max - 2 kb - kc columns (or k_ro), and the result
    still equals the dense eigendecomposition."""
    n = 1800
    e, _ = synth.sbm(n, 12, d_in=20, d_out=4, uneven=True, seed=1)
    g = oracle_mod.build_csr(e, n)
    p = oracle_mod.Params(k_want=12, kb=3, m=11, seed=1, act_max=15, dim_max=21, k_ro=k_ro)
    r = oracle_mod.bchdav(g, p)
    _check_common(oracle_mod, g, r, 12)
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(g))
    assert np.abs(r.evals - lam[:12]).max() <= 1e-10
    h = r.history
    fired = [i for i, x in enumerate(h) if x["outer_restart"]]
    assert fired
    for i in fired:
        kc_after = h[i]["kc"] + h[i]["ec"] - h[i]["n_unlocked"]
        ro = 21 - 2 * 3 - kc_after
        if k_ro:
            ro = min(ro, k_ro)
        # the next iteration starts from the cut active block plus one new block
        assert h[i + 1]["kact"] == ro + 3 and h[i + 1]["kc"] == kc_after
        assert h[i]["ksub"] - h[i]["n_unlocked"] + 3 > 21


def test_exit_certificate_unlocks_and_refines(oracle_mod):
    """Exit certificate (fresh residuals of the returned pairs): with a stricter
    certificate tolerance than the loop's, the pairs that fail it are un-locked
    and filtered again until every fresh residual meets it."""
    n = 1500
    e, _ = synth.sbm(n, 4, d_in=16, d_out=3, uneven=True, seed=5)
    g = oracle_mod.build_csr(e, n)
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(g))
    plain = oracle_mod.bchdav(g, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1))
    r = oracle_mod.bchdav(g, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1, certify_tol=1e-13))
    assert plain.n_unlocked == 0 and plain.max_residual > 1e-13
    assert r.status == "ok" and r.n_unlocked > 0 and r.iterations > plain.iterations
    R = oracle_mod.apply_laplacian(g, np.asfortranarray(r.evecs)) - r.evecs * r.evals
    assert np.sqrt((R * R).sum(0)).max() <= 1e-13
    assert np.abs(r.evals - lam[:4]).max() <= 1e-12
    # a certificate that cannot be met ends unconverged after refine_sweeps rounds
    bad = oracle_mod.bchdav(g, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1, certify_tol=1e-30,
                                                 refine_sweeps=2))
    assert bad.status == "certificate" and bad.certified < 4
    assert sum(1 for x in bad.history if x["n_unlocked"]) == 2
