"""GPU parity for the Householder TSQR (Sec. 3.3) against the oracle's flat
Householder QR, element by element (both with a non-negative diagonal of R,
which makes the thin QR unique): shapes that span one chunk, several chunks
with a ragged tail, several tree levels, in place; rank-deficient blocks by
their invariants; the orthonormalizer and the solver with TSQR in place of
Cholesky QR against the oracle's DGKS and Davidson.

Tolerance: Householder QR is backward stable, so the factors of a matrix with
condition number kappa agree to O(kappa * eps) (Q) and O(kappa * eps * ||X||)
(R); the bound used is 64 * kappa * eps times those scales."""

import numpy as np
import pytest

import synth
from conftest import sin_max_angle

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _gpu_tsqr(cd, X, in_place=False):
    import torch
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Q, R = cd.tsqr(Xt, Q=Xt if in_place else None)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), R.cpu().numpy()


def _check_parity(tq, X, Q, R):
    Qo, Ro = tq.householder_qr(X)
    kappa = np.linalg.cond(X)
    nx = np.linalg.norm(X, 2)
    dq, dr = np.max(np.abs(Q - Qo)), np.max(np.abs(R - Ro))
    print("  kappa %.3g  max|dQ| %.3g  max|dR|/||X|| %.3g" % (kappa, dq, dr / nx), flush=True)
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0.0)
    assert dq <= 64 * kappa * EPS
    assert dr <= 64 * kappa * EPS * nx


@pytest.fixture(scope="module")
def tq(oracle_mod):
    from oracle import tsqr
    return tsqr


# (n, kb): one chunk, exactly one chunk, ragged tails, n == kb, several tree levels
SHAPES = [(1, 1), (4, 4), (100, 1), (255, 8), (256, 32), (257, 32), (1000, 33), (5000, 64), (20_011, 17),
          (100_000, 5), (64, 64), (65, 64), (3000, 9)]


@pytest.mark.parametrize("n,kb", SHAPES)
def test_tsqr_parity(cd, tq, dev, n, kb):
    X = np.random.default_rng(n * 131 + kb).standard_normal((n, kb))
    print("case tsqr n=%d kb=%d" % (n, kb), flush=True)
    Q, R = _gpu_tsqr(cd, X)
    _check_parity(tq, X, Q, R)


def test_tsqr_in_place_and_scaled_columns(cd, tq, dev):
    X = np.random.default_rng(3).standard_normal((7000, 24)) * np.logspace(-3, 3, 24)
    print("case tsqr in place n=7000 kb=24", flush=True)
    Q, R = _gpu_tsqr(cd, X, in_place=True)
    _check_parity(tq, X, Q, R)


def test_tsqr_full_size_sbm200k_block(cd, tq, dev):
    X = np.random.default_rng(4).standard_normal((200_000, 32))
    print("case tsqr n=200000 kb=32", flush=True)
    Q, R = _gpu_tsqr(cd, X)
    _check_parity(tq, X, Q, R)


def test_tsqr_full_size_2m_invariants(cd, dev):
    """2M x 64 (the FP32-form workload's block): invariants, and R against the
    Cholesky factor of the Gram matrix (well conditioned, so close)."""
    X = np.random.default_rng(5).standard_normal((2_000_000, 64))
    print("case tsqr n=2000000 kb=64", flush=True)
    Q, R = _gpu_tsqr(cd, X)
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
    assert np.linalg.norm(Q.T @ Q - np.eye(64), 2) <= 64 * 64 * EPS
    assert np.linalg.norm(Q @ R - X) <= 64 * 64 * EPS * np.linalg.norm(X)
    L = np.linalg.cholesky(X.T @ X)
    assert np.max(np.abs(R - L.T)) <= 1e-10 * np.linalg.norm(X, 2)


def test_tsqr_rank_deficient(cd, dev):
    X = np.random.default_rng(6).standard_normal((3000, 8))
    X[:, 3] = X[:, 0] - 0.5 * X[:, 1]
    X[:, 6] = 0.0
    print("case tsqr rank deficient n=3000 kb=8", flush=True)
    Q, R = _gpu_tsqr(cd, X)
    assert np.linalg.norm(Q.T @ Q - np.eye(8), 2) <= 100 * EPS
    assert np.linalg.norm(Q @ R - X) <= 100 * EPS * np.linalg.norm(X)
    assert abs(R[3, 3]) <= 1e-12 * np.linalg.norm(X, 2)
    assert np.all(R[:, 6] == 0.0)


def test_tsqr_errors(cd, dev):
    import torch
    X = torch.zeros((10, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(cd.ChebdavError):
        cd.tsqr(X)
    X = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(cd.ChebdavError):
        cd.tsqr(X)


def _basis(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return np.ascontiguousarray(q)


@pytest.mark.parametrize("n,ksub,kb", [(2000, 40, 8), (50_000, 224, 32), (100_000, 384, 64)])
def test_orthonormalize_tsqr_matches_dgks(cd, oracle_mod, dev, n, ksub, kb):
    """Gram-Schmidt of a full-rank block and its QR give the same columns."""
    import torch
    V = _basis(n, ksub, 0)
    X = np.random.default_rng(1).standard_normal((n, kb))
    print("case orth tsqr n=%d ksub=%d kb=%d" % (n, ksub, kb), flush=True)
    Xt = torch.from_numpy(X.copy()).cuda()
    rep = cd.orthonormalize(torch.from_numpy(V).cuda(), Xt, method="tsqr")
    Q = Xt.cpu().numpy()
    Qo, rep_o, _ = oracle_mod.dgks(np.asfortranarray(V), X.copy(), seed=0, next_col=0)
    assert rep == rep_o == 0
    assert np.max(np.abs(Q - Qo)) <= 1e-12
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 10 * ksub * EPS


def test_orthonormalize_tsqr_dependent_columns(cd, oracle_mod, dev):
    import torch
    n, kb = 1500, 6
    V = _basis(n, 10, 8)
    X = np.random.default_rng(9).standard_normal((n, kb))
    X[:, 2] = X[:, 0]
    X[:, 4] = V @ np.arange(1.0, 11.0)
    X[:, 5] = 0.0
    Xt = torch.from_numpy(X.copy()).cuda()
    rep = cd.orthonormalize(torch.from_numpy(V).cuda(), Xt, seed=2, first_random_col=100, method="tsqr")
    Q = Xt.cpu().numpy()
    _, rep_oracle, _ = oracle_mod.dgks(np.asfortranarray(V), X.copy(), seed=2, next_col=100)
    assert rep == rep_oracle == 3
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 100 * EPS
    keep = X[:, [0, 1, 3]] - V @ (V.T @ X[:, [0, 1, 3]])
    assert np.linalg.norm(keep - Q @ (Q.T @ keep)) <= 1e-12 * np.linalg.norm(keep)


@pytest.mark.parametrize("config,k,kb,m", [("sbm5k", 4, 4, 11), ("sbm200k", 32, 32, 15)])
def test_solve_with_tsqr(cd, oracle_mod, dev, config, k, kb, m):
    import torch
    e, n, _ = synth.make_config_graph(config)
    print("case solve tsqr %s" % config, flush=True)
    o = oracle_mod.build_csr(e, n)
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=k, kb=kb, m=m, seed=1))
    g = cd.build_laplacian(e, n)
    r = cd.solve(g, cd.make_params(k_want=k, kb=kb, m=m, seed=1, orth="tsqr"))
    ev, V = r.evals.cpu().numpy(), r.evecs.cpu().numpy()
    R = oracle_mod.apply_laplacian(o, np.asfortranarray(V)) - V * ev
    res = np.sqrt((R * R).sum(0))
    print("  iters gpu %d oracle %d; max res %.3g; max dlam %.3g" %
          (r.stats["iterations"], ref.iterations, res.max(), np.abs(ev - ref.evals).max()), flush=True)
    assert res.max() <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert np.linalg.norm(V.T @ V - np.eye(k), 2) <= 1e-12
    assert sin_max_angle(ref.evecs, V) <= 1e-6
    assert abs(r.stats["iterations"] - ref.iterations) <= 2
    del g
    torch.cuda.synchronize()
