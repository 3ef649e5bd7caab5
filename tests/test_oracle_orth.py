"""Pins for the oracle's DGKS orthonormalization: orthonormality, orthogonality
to the basis, the span it must reach, and replacement of exactly dependent
columns (the only case whose count is fixed independently of the threshold)."""

import numpy as np

EPS = np.finfo(np.float64).eps


def _basis(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return np.asfortranarray(q)


def test_invariants_and_span(oracle_mod):
    n, ksub, kb = 2000, 40, 8
    V = _basis(n, ksub, 0)
    X = np.random.default_rng(1).standard_normal((n, kb))
    Q, nrep, nxt = oracle_mod.dgks(V, X, seed=3, next_col=10)
    assert nrep == 0 and nxt == 10
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 10 * ksub * EPS
    # span(Q) = span((I - V V^T) X): projecting X's remainder onto Q loses nothing
    Xp = X - V @ (V.T @ X)
    resid = Xp - Q @ (Q.T @ Xp)
    assert np.linalg.norm(resid) <= 1e-12 * np.linalg.norm(Xp)
    # Gram-Schmidt order: column j of Q lies in span of the first j+1 columns
    for j in range(kb):
        B = np.concatenate([V, Xp[:, : j + 1]], axis=1)
        coef = np.linalg.lstsq(B, Q[:, j], rcond=None)[0]
        assert np.linalg.norm(B @ coef - Q[:, j]) < 1e-10


def test_ill_conditioned_block(oracle_mod):
    n, kb = 3000, 6
    V = _basis(n, 20, 4)
    base = np.random.default_rng(5).standard_normal((n, 1))
    X = base + 1e-7 * np.random.default_rng(6).standard_normal((n, kb))   # kappa ~ 1e7
    X = X + V @ np.random.default_rng(7).standard_normal((20, kb)) * 1e3  # mostly in span(V)
    Q, nrep, _ = oracle_mod.dgks(V, X, seed=1, next_col=0)
    assert nrep == 0
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 100 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 100 * 20 * EPS


def test_exactly_dependent_columns_replaced(oracle_mod):
    n, kb = 1500, 6
    V = _basis(n, 10, 8)
    X = np.random.default_rng(9).standard_normal((n, kb))
    X[:, 2] = X[:, 0]                      # duplicate of a new column
    X[:, 4] = V @ np.arange(1.0, 11.0)     # exactly inside span(V)
    X[:, 5] = 0.0                          # zero column
    Q, nrep, nxt = oracle_mod.dgks(V, X, seed=2, next_col=100)
    assert nrep == 3 and nxt == 103
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 100 * EPS
    # the replacement for column 2 is Philox column 100, orthogonalized
    r = oracle_mod.random_block(2, n, [100])[:, 0]
    B = np.concatenate([V, Q[:, :2]], axis=1)
    rp = r - B @ (B.T @ r)
    assert abs(abs(Q[:, 2] @ rp) - np.linalg.norm(rp)) < 1e-10 * np.linalg.norm(rp)


def test_no_basis(oracle_mod):
    X = np.random.default_rng(0).standard_normal((300, 4))
    Q, nrep, _ = oracle_mod.dgks(np.zeros((300, 0)), X, seed=0, next_col=0)
    assert nrep == 0 and np.linalg.norm(Q.T @ Q - np.eye(4)) < 1e-14
