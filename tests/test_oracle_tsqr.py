"""Pins for the oracle's tall-skinny QR (Sec. 3.3, distributed orthonormalization
by TSQR): a hand-computed exact factorization, LAPACK's Householder QR with the
same sign convention, the Cholesky factor of X^T X, orthogonal-column and
rank-deficient closed forms, and the paper's tree (any leaf count and fan-in)
against the flat factorization."""

import numpy as np
import pytest

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def tq(oracle_mod):
    from oracle import tsqr
    return tsqr


def test_exact_small(tq):
    # [[3, 2], [4, 11]] = [[.6, -.8], [.8, .6]] [[5, 10], [0, 5]], worked by hand
    X = np.array([[3.0, 2.0], [4.0, 11.0], [0.0, 0.0]])
    Q, R = tq.householder_qr(X)
    np.testing.assert_allclose(R, [[5.0, 10.0], [0.0, 5.0]], atol=1e-14)
    np.testing.assert_allclose(Q, [[0.6, -0.8], [0.8, 0.6], [0.0, 0.0]], atol=1e-15)
    Q, R = tq.householder_qr(np.array([[3.0], [4.0]]))
    np.testing.assert_allclose(R, [[5.0]], atol=1e-15)
    np.testing.assert_allclose(Q[:, 0], [0.6, 0.8], atol=1e-16)
    # a negative leading entry: R's diagonal stays non-negative, Q takes the sign
    Q, R = tq.householder_qr(np.array([[-3.0], [4.0]]))
    np.testing.assert_allclose(R, [[5.0]], atol=1e-15)
    np.testing.assert_allclose(Q[:, 0], [-0.6, 0.8], atol=1e-16)


@pytest.mark.parametrize("n,k,seed", [(5, 5, 0), (40, 7, 1), (300, 32, 2), (1000, 64, 3)])
def test_matches_lapack(tq, n, k, seed):
    X = np.random.default_rng(seed).standard_normal((n, k))
    Q, R = tq.householder_qr(X)
    Ql, Rl = np.linalg.qr(X)
    s = np.where(np.diag(Rl) < 0, -1.0, 1.0)
    Ql, Rl = Ql * s, Rl * s[:, None]
    kappa = np.linalg.cond(X)
    assert np.max(np.abs(R - Rl)) <= 50 * kappa * EPS * np.linalg.norm(X, 2)
    assert np.max(np.abs(Q - Ql)) <= 50 * kappa * EPS
    # R^T R = X^T X: R is the transposed Cholesky factor of the Gram matrix
    L = np.linalg.cholesky(X.T @ X)
    assert np.max(np.abs(R - L.T)) <= 100 * kappa * kappa * EPS * np.linalg.norm(X, 2)


@pytest.mark.parametrize("n,k", [(50, 3), (2000, 17)])
def test_invariants(tq, n, k):
    X = np.random.default_rng(n).standard_normal((n, k)) * np.logspace(0, 6, k)
    Q, R = tq.householder_qr(X)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.all(np.diag(R) >= 0)
    assert np.linalg.norm(Q.T @ Q - np.eye(k), 2) <= 10 * k * EPS
    assert np.linalg.norm(Q @ R - X) <= 10 * k * EPS * np.linalg.norm(X)


def test_orthogonal_columns(tq):
    U, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((500, 6)))
    s = np.array([3.0, 1.0, 0.5, 7.0, 2.0, 1e-3])
    Q, R = tq.householder_qr(U * s)
    np.testing.assert_allclose(R, np.diag(s), atol=1e-13)
    sign = np.sign(np.sum(Q * U, axis=0))
    np.testing.assert_allclose(Q, U * sign, atol=1e-13)
    assert np.all(sign == 1.0)


def test_rank_deficient(tq):
    X = np.random.default_rng(5).standard_normal((200, 5))
    X[:, 2] = 2.0 * X[:, 0] - X[:, 1]
    X[:, 4] = 0.0
    Q, R = tq.householder_qr(X)
    assert np.linalg.norm(Q.T @ Q - np.eye(5), 2) <= 100 * EPS
    assert np.linalg.norm(Q @ R - X) <= 100 * EPS * np.linalg.norm(X)
    assert abs(R[2, 2]) <= 1e-13 * np.linalg.norm(X)
    assert R[4, 4] == 0.0 and np.all(R[:, 4] == 0.0)


@pytest.mark.parametrize("n,k,p,q", [(1000, 8, 4, 2), (1000, 8, 4, 4), (3001, 16, 9, 4), (777, 5, 7, 3),
                                     (64, 8, 8, 2)])
def test_tree_equals_flat(tq, n, k, p, q):
    X = np.random.default_rng(n + k).standard_normal((n, k))
    Qf, Rf = tq.householder_qr(X)
    Qt, Rt = tq.tsqr_tree(X, p, q)
    assert np.max(np.abs(Rt - Rf)) <= 1e-12 * np.linalg.norm(X, 2)
    assert np.max(np.abs(Qt - Qf)) <= 1e-12


def test_tree_on_paper_example(tq):
    # the four-process, fan-in-two example of Sec. 3.3: R_0123 is the R of V
    X = np.random.default_rng(11).standard_normal((400, 6))
    _, Rf = tq.householder_qr(X)
    Q0123, R0123 = tq.tsqr_tree(X, 4, 2)
    assert np.max(np.abs(R0123 - Rf)) <= 1e-12 * np.linalg.norm(X, 2)
    assert np.linalg.norm(Q0123 @ R0123 - X) <= 1e-12 * np.linalg.norm(X)


def test_planted_mistakes_fail(tq):
    """Mistakes a QR can make are caught by the checks above: a reflector applied
    with the wrong sign, a dropped row, a transposed R."""
    X = np.random.default_rng(12).standard_normal((60, 4))
    Q, R = tq.householder_qr(X)
    assert np.linalg.norm(Q @ R.T - X) > 1e-3
    Qb = Q.copy()
    Qb[:, 1] *= -1.0
    assert np.linalg.norm(Qb @ R - X) > 1e-3
    Rb = R.copy()
    Rb[1, 2] = 0.0
    assert np.linalg.norm(Q @ Rb - X) > 1e-6
