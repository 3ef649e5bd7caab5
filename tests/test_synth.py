"""Synthetic workload generators: reproducibility and the properties each
workload is specified by (sizes, degrees, simplicity, connectivity)."""

import math

import numpy as np

import synth
from synth.graphs import _bernoulli_positions, _unrank_upper


def _is_simple(edges, n):
    assert edges.dtype == np.int64 and edges.ndim == 2 and edges.shape[1] == 2
    assert (edges[:, 0] < edges[:, 1]).all()
    assert edges.min() >= 0 and edges.max() < n
    key = edges[:, 0] * n + edges[:, 1]
    assert np.unique(key).size == key.size


def test_unrank_upper_exhaustive():
    for n in [2, 3, 7, 64]:
        i, j = _unrank_upper(np.arange(n * (n - 1) // 2), n)
        ri, rj = np.triu_indices(n, 1)
        assert (i == ri).all() and (j == rj).all()


def test_unrank_upper_large_n_edges():
    n = 8_000_000
    total = n * (n - 1) // 2
    idx = np.array([0, 1, n - 2, n - 1, total - 3, total - 2, total - 1], dtype=np.int64)
    i, j = _unrank_upper(idx, n)
    off = i * (2 * n - i - 1) // 2
    assert (idx == off + (j - i - 1)).all()
    assert (i < j).all() and (j < n).all()


def test_bernoulli_positions_rate():
    rng = np.random.Generator(np.random.PCG64(5))
    m, p = 2_000_000, 0.01
    pos = _bernoulli_positions(rng, m, p)
    assert (np.diff(pos) > 0).all() and pos.min() >= 0 and pos.max() < m
    assert abs(pos.size - m * p) < 5 * math.sqrt(m * p)


def test_sbm_reproducible_and_shaped():
    e1, l1 = synth.sbm(5000, 4, p_in=0.016, p_out=0.0008, seed=11)
    e2, l2 = synth.sbm(5000, 4, p_in=0.016, p_out=0.0008, seed=11)
    assert np.array_equal(e1, e2) and np.array_equal(l1, l2)
    _is_simple(e1, 5000)
    assert np.bincount(l1).tolist() == [1250] * 4
    # expected degree 0.016 * 1249 + 0.0008 * 3750 = 22.98
    mean_deg = 2 * len(e1) / 5000
    assert abs(mean_deg - 22.98) < 0.5
    intra = (l1[e1[:, 0]] == l1[e1[:, 1]]).mean()
    assert abs(intra - 19.984 / 22.984) < 0.02


def test_sbm_uneven_degrees():
    n, b = 100_000, 16
    e, lab = synth.sbm(n, b, d_in=20.0, d_out=4.0, uneven=True, seed=3)
    _is_simple(e, n)
    sizes = np.bincount(lab)
    assert sizes.sum() == n and sizes.min() > 0
    assert sizes.max() / sizes.min() < 2.05
    deg = np.bincount(e.ravel(), minlength=n)
    assert abs(deg.mean() - 24.0) < 0.3


def test_block_sizes_sum():
    for n, b in [(200_000, 32), (2_000_000, 64), (17, 5)]:
        s = synth.sbm_block_sizes(n, b, True, 9)
        assert s.sum() == n and len(s) == b


def test_chung_lu_lcc_connected():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    e, n = synth.chung_lu(50_000, seed=4)
    _is_simple(e, n)
    a = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    assert connected_components(a, directed=False)[0] == 1
    deg = np.bincount(e.ravel(), minlength=n)
    assert deg.min() >= 1
    assert deg.max() <= 3 * math.sqrt(50_000)
    w = synth.chung_lu_weights(50_000, 2.1, 16.0, math.sqrt(50_000))
    assert abs(w.mean() - 16.0) < 1e-6 and w.max() <= math.sqrt(50_000) + 1e-9


def test_closed_form_graphs():
    _is_simple(synth.cycle_graph(10), 10)
    assert len(synth.cycle_graph(10)) == 10
    assert len(synth.path_graph(10)) == 9
    assert len(synth.complete_graph(6)) == 15
    assert len(synth.complete_bipartite_graph(3, 4)) == 12
    assert len(synth.hypercube_graph(4)) == 32
    e, n = synth.disjoint_union([(synth.cycle_graph(5), 5), (synth.path_graph(3), 3)])
    assert n == 8 and len(e) == 7 and e.max() == 7
