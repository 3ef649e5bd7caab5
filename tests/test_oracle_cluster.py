"""Pins for the oracle's clustering tail (Alg. 1, steps 3-4): the agreement
scores against brute-force pair counting and exact cases, K-means against its
fixed-point conditions and planted clusters, and the whole tail on an SBM
graph's exact eigenvectors (dense eigh) against the planted blocks."""

import itertools
import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def cl(oracle_mod):
    from oracle import cluster
    return cluster


def _ari_pairs(a, b):
    """Adjusted Rand index by counting every pair (Hubert & Arabie's definition)."""
    n = len(a)
    both = same_a = same_b = 0
    for i, j in itertools.combinations(range(n), 2):
        sa, sb = a[i] == a[j], b[i] == b[j]
        both += sa and sb
        same_a += sa
        same_b += sb
    pairs = n * (n - 1) / 2
    exp = same_a * same_b / pairs
    mx = (same_a + same_b) / 2
    return (both - exp) / (mx - exp)


def _nmi_def(a, b):
    """NMI from the joint distribution written out entry by entry."""
    n = len(a)
    la, lb = sorted(set(a)), sorted(set(b))
    pa = {x: sum(1 for v in a if v == x) / n for x in la}
    pb = {y: sum(1 for v in b if v == y) / n for y in lb}
    mi = 0.0
    for x in la:
        for y in lb:
            pxy = sum(1 for u, v in zip(a, b) if u == x and v == y) / n
            if pxy > 0:
                mi += pxy * math.log(pxy / (pa[x] * pb[y]))
    ha = -sum(p * math.log(p) for p in pa.values())
    hb = -sum(p * math.log(p) for p in pb.values())
    return mi / math.sqrt(ha * hb)


def test_scores_against_brute_force(cl):
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(5, 40))
        a = rng.integers(0, int(rng.integers(2, 6)), n)
        b = rng.integers(0, int(rng.integers(2, 6)), n)
        if len(set(a)) < 2 or len(set(b)) < 2:
            continue
        assert abs(cl.ari(a, b) - _ari_pairs(a, b)) < 1e-12
        assert abs(cl.nmi(a, b) - _nmi_def(a, b)) < 1e-12


def test_scores_exact_cases(cl):
    a = np.repeat(np.arange(4), 25)
    perm = np.array([2, 0, 3, 1])
    assert cl.ari(a, perm[a]) == 1.0            # same partition, other names
    assert abs(cl.nmi(a, perm[a]) - 1.0) < 1e-15
    # a = i mod 2 and b = (i // 2) mod 2 are independent on 4m points: I(a; b) = 0
    i = np.arange(400)
    assert abs(cl.nmi(i % 2, (i // 2) % 2)) < 1e-15
    # ARI of two such independent balanced partitions: sum_ij C(100,2) vs expectation
    assert cl.ari(i % 2, (i // 2) % 2) < 0.0


def test_row_normalize(cl):
    U = np.random.default_rng(1).standard_normal((50, 6))
    U[7] = 0.0
    F = cl.row_normalize(U)
    nr = np.sqrt((F * F).sum(1))
    assert np.abs(np.delete(nr, 7) - 1.0).max() < 1e-15
    assert (F[7] == 0.0).all()


def test_kmeans_recovers_separated_clusters(cl):
    rng = np.random.default_rng(2)
    K, k = 6, 5
    centres = 10.0 * rng.standard_normal((K, k))
    truth = rng.integers(0, K, 600)
    F = centres[truth] + 0.05 * rng.standard_normal((600, k))
    labels, C, rounds, inertia = cl.kmeans(F, K, seed=3)
    assert cl.ari(labels, truth) == 1.0
    # fixed point: centres are the member means, every row at its nearest centre
    for c in range(K):
        assert np.abs(C[c] - F[labels == c].mean(0)).max() < 1e-12
    D = ((F[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    assert (labels == D.argmin(1)).all()
    assert abs(inertia - D.min(1).sum()) < 1e-9 * inertia


def test_kmeans_single_cluster_and_inertia_monotone(cl):
    F = np.random.default_rng(4).standard_normal((300, 3))
    labels, C, _, inertia = cl.kmeans(F, 1, seed=0)
    assert (labels == 0).all()
    assert np.abs(C[0] - F.mean(0)).max() < 1e-14
    # Lloyd never increases the objective: rerun with growing round limits
    vals = [cl.kmeans(F, 7, seed=1, max_iter=r)[3] for r in (1, 2, 3, 5, 8, 50)]
    assert all(vals[i + 1] <= vals[i] * (1 + 1e-12) for i in range(len(vals) - 1))


def test_farthest_first(cl):
    # points on a line: after any start, the next centre is the farther end
    F = np.arange(10, dtype=np.float64)[:, None]
    idx = cl.farthest_first(F, 3, seed=5)
    f = idx[0]
    assert idx[1] == (9 if f < 4.5 else 0)
    assert 0 <= cl.first_index(10, 5) < 10
    assert cl.first_index(10**12, 7) < 10**12


def test_spectral_tail_on_planted_blocks(cl, oracle_mod):
    """Exact eigenvectors of a strongly planted SBM: the tail recovers the blocks."""
    e, truth = synth.sbm(400, 4, p_in=0.2, p_out=0.005, seed=9)
    g = oracle_mod.build_csr(e, 400)
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(g))
    F = cl.row_normalize(Q[:, :4])
    labels, *_ = cl.kmeans(F, 4, seed=1)
    assert cl.ari(labels, truth) == 1.0
    assert abs(cl.nmi(labels, truth) - 1.0) < 1e-12
