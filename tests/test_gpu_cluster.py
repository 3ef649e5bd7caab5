"""GPU: the clustering tail (row normalization + K-means, chebdav_cluster)
against the oracle's FP64 restatement on the same inputs, its edge cases, and
the whole spectral-clustering pipeline on planted SBM graphs.

Bar: labels identical to the oracle's (both sides take every nearest-centre
decision in FP64 with the same coordinate order; the row sums behind the
centres differ only in their summation order, so a label could differ only for
a row equidistant from two centres to rounding, which these inputs do not
have), centres within 1e-12 absolute, equal round counts, inertia within
1e-10 relative."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ocl(oracle_mod):
    from oracle import cluster
    return cluster


def _compare(cd, ocl, U, K, seed, max_iter=100):
    import torch
    Ut = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    labels, C, rounds, inertia = cd.cluster(Ut, K, seed=seed, max_iter=max_iter)
    labels, C = labels.cpu().numpy(), C.cpu().numpy()
    F = ocl.row_normalize(U)
    wl, wC, wr, wi = ocl.kmeans(F, K, seed=seed, max_iter=max_iter)
    assert np.array_equal(labels, wl)
    assert np.abs(C - wC).max() <= 1e-12
    assert rounds == wr
    assert abs(inertia - wi) <= 1e-10 * max(wi, 1e-300)
    return labels, C, rounds, inertia


@pytest.mark.parametrize("n,k,K,seed", [(5000, 8, 8, 1), (3001, 5, 3, 2), (20000, 32, 32, 3), (777, 64, 10, 4),
                                        (4096, 1, 2, 5), (1000, 16, 1, 6)])
def test_cluster_matches_oracle(cd, ocl, dev, n, k, K, seed):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((K, k))
    if k == 1:  # one coordinate normalizes to +-1: keep both signs present
        centres = np.where(np.arange(K)[:, None] % 2 == 0, 1.0, -1.0)
    truth = rng.integers(0, K, n)
    U = centres[truth] * rng.uniform(0.5, 2.0, (n, 1)) + 0.05 * rng.standard_normal((n, k))
    print("case cluster n=%d k=%d K=%d" % (n, k, K), flush=True)
    _compare(cd, ocl, U, K, seed)


def test_cluster_zero_rows_duplicates_and_round_limit(cd, ocl, dev):
    rng = np.random.default_rng(7)
    U = rng.standard_normal((600, 6))
    U[::50] = 0.0                   # zero rows stay zero and form their own group
    U[1::7] = U[1]                  # many identical rows
    _compare(cd, ocl, U, 5, seed=3)
    _compare(cd, ocl, U, 5, seed=3, max_iter=1)
    _compare(cd, ocl, U, 5, seed=3, max_iter=2)


def test_cluster_every_row_its_own_centre(cd, ocl, dev):
    U = np.random.default_rng(8).standard_normal((40, 3))
    labels, C, rounds, inertia = _compare(cd, ocl, U, 40, seed=1)
    assert len(set(labels.tolist())) == 40 and inertia <= 1e-28


def test_cluster_errors(cd, dev):
    import torch
    U = torch.zeros(10, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(cd.ChebdavError):
        cd.cluster(U, 11)                            # more clusters than rows
    with pytest.raises(cd.ChebdavError):
        cd.cluster(torch.zeros(10, 65, dtype=torch.float64, device="cuda"), 2)   # k > 64
    with pytest.raises(cd.ChebdavError):
        cd.cluster(U, 2, max_iter=0)


def test_cluster_deterministic(cd, dev):
    import torch
    U = torch.randn(50_000, 16, dtype=torch.float64, device="cuda")
    a = cd.cluster(U, 16, seed=2)
    b = cd.cluster(U, 16, seed=2)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and a[2:] == b[2:]


@pytest.mark.parametrize("workload", ["sbm5k", "sbm200k"])
def test_spectral_pipeline(cd, ocl, dev, workload):
    """Graph -> eigenvectors (GPU solver) -> clustering tail: the tail agrees with
    the oracle's on the GPU eigenvectors, and the partition recovers the planted
    blocks (ARI and NMI reported; the bar is the oracle's own score on the same
    vectors, which the identical labels imply)."""
    from paper_2212_04443_amd import spectral
    e, n, cfg = synth.make_config_graph(workload)
    g = cd.build_laplacian(e, n)
    out = spectral.spectral_clustering(g, cfg["k"], kb=cfg["kb"], m=cfg["m"], seed=1)
    U = out["evecs"].cpu().numpy()
    labels = out["labels"].cpu().numpy()
    wl, *_ = ocl.kmeans(ocl.row_normalize(U), cfg["k"], seed=1)
    assert np.array_equal(labels, wl)
    truth = cfg["labels"]
    a, m = spectral.adjusted_rand_index(labels, truth), spectral.normalized_mutual_info(labels, truth)
    print("%s: ARI %.4f NMI %.4f, %d K-means rounds, solve %.1f ms, cluster %.1f ms"
          % (workload, a, m, out["rounds"], 1e3 * out["solve_s"], 1e3 * out["cluster_s"]))
    assert abs(a - ocl.ari(labels, truth)) < 1e-12 and abs(m - ocl.nmi(labels, truth)) < 1e-12
