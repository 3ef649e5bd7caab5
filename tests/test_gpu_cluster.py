"""GPU: the clustering tail (row normalization + K-means, chebdav_cluster)
against the oracle's FP64 restatement on the same inputs, its edge cases, and
the whole spectral-clustering pipeline on planted SBM graphs.

Bar: labels identical to the oracle's, except at a row that is equidistant from
the two centres concerned to rounding (relative gap of the squared distances
<= 1e-12): the row norms and centre sums are rounded differently on the two
sides, so such a tie may be broken either way, and the K-means rounds after it
then legitimately follow another path.  With identical labels: centres within
1e-12 absolute, equal round counts, inertia within 1e-10 relative.  After a
tie: the GPU's own result must be consistent (each centre the mean of its rows
within 1e-12, every row at a nearest centre up to a tie, inertia the sum of its
squared distances within 1e-10)."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TIE_GAP = 1e-12


@pytest.fixture(scope="module")
def ocl(oracle_mod):
    from oracle import cluster
    return cluster


def _dist_table(ocl, F, C):
    return np.stack([ocl.sq_dist(F, C[c]) for c in range(C.shape[0])], axis=1)


def _ties_only(D, a, b):
    """Rows where labels a and b differ are ties under the distance table D."""
    rows = np.nonzero(a != b)[0]
    da, db = D[rows, a[rows]], D[rows, b[rows]]
    gap = np.abs(da - db) / np.maximum(np.maximum(da, db), 1e-300)
    return bool((gap <= TIE_GAP).all()), rows


def _compare(cd, ocl, U, K, seed, max_iter=100):
    import torch
    Ut = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    labels, C, rounds, inertia = cd.cluster(Ut, K, seed=seed, max_iter=max_iter)
    labels, C = labels.cpu().numpy(), C.cpu().numpy()
    F = ocl.row_normalize(U)
    wl, wC, wr, wi = ocl.kmeans(F, K, seed=seed, max_iter=max_iter)
    if np.array_equal(labels, wl):
        assert np.abs(C - wC).max() <= 1e-12
        assert rounds == wr
        assert abs(inertia - wi) <= 1e-10 * max(wi, 1e-300)
        return labels, C, rounds, inertia
    # a tie was broken the other way: the final labels may differ only at ties,
    # and the GPU's result must be a consistent K-means state of its own
    ok, rows = _ties_only(_dist_table(ocl, F, wC), labels, wl)
    print("labels differ from the oracle's at %d rows (ties: %s)" % (len(rows), ok))
    assert ok
    D = _dist_table(ocl, F, C)
    for c in range(K):
        mem = labels == c
        if mem.any():
            assert np.abs(C[c] - F[mem].sum(axis=0) / mem.sum()).max() <= 1e-12
    if rounds < max_iter:
        best = D.min(axis=1)
        mine = D[np.arange(len(labels)), labels]
        assert ((mine - best) <= TIE_GAP * np.maximum(mine, 1e-300)).all()
    want = float(D[np.arange(len(labels)), labels].sum())
    assert abs(inertia - want) <= 1e-10 * max(want, 1e-300)
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
    blocks (ARI and NMI reported, and recomputed by the oracle's own scores)."""
    from paper_2212_04443_amd import spectral
    e, n, cfg = synth.make_config_graph(workload)
    g = cd.build_laplacian(e, n)
    out = spectral.spectral_clustering(g, cfg["k"], kb=cfg["kb"], m=cfg["m"], seed=1)
    U = out["evecs"].cpu().numpy()
    labels = out["labels"].cpu().numpy()
    F = ocl.row_normalize(U)
    wl, wC, *_ = ocl.kmeans(F, cfg["k"], seed=1)
    assert _ties_only(_dist_table(ocl, F, wC), labels, wl)[0]
    truth = cfg["labels"]
    a, m = spectral.adjusted_rand_index(labels, truth), spectral.normalized_mutual_info(labels, truth)
    print("%s: ARI %.4f NMI %.4f, %d K-means rounds, solve %.1f ms, cluster %.1f ms"
          % (workload, a, m, out["rounds"], 1e3 * out["solve_s"], 1e3 * out["cluster_s"]))
    assert abs(a - ocl.ari(labels, truth)) < 1e-12 and abs(m - ocl.nmi(labels, truth)) < 1e-12
