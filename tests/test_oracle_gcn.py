"""Pins for the oracle's warm-start network: hand-derived gradients against
central finite differences (FP64), and the loss's invariances and extreme values."""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def small(oracle_mod):
    from oracle import gcn
    e, _ = synth.sbm(160, 4, p_in=0.12, p_out=0.01, seed=3)
    csr = oracle_mod.build_csr(e, 160)
    dims = (5, 7, 6, 4)
    W = gcn.glorot(11, dims)
    X0 = np.random.default_rng(2).standard_normal((160, dims[0]))
    lam, Q = np.linalg.eigh(oracle_mod.dense_laplacian(csr))
    U = Q[:, :4]
    return gcn, csr, dims, W, X0, U


def _total_loss(gcn, csr, X0, W, U):
    out, _ = gcn.forward(csr, X0, W)
    return gcn.subspace_loss(out, U)[0]


def test_ahat_is_identity_minus_laplacian(oracle_mod, small):
    gcn, csr, *_ = small
    X = np.random.default_rng(0).standard_normal((160, 3))
    A = oracle_mod.dense_laplacian(csr)
    assert np.abs(gcn.ahat(csr, X) - (np.eye(160) - A) @ X).max() < 1e-13


def test_loss_gradient_finite_differences(small):
    gcn, csr, dims, W, X0, U = small
    X = np.random.default_rng(5).standard_normal((160, 4))
    L, dX = gcn.subspace_loss(X, U)
    h = 1e-6
    rng = np.random.default_rng(6)
    for _ in range(12):
        i, j = rng.integers(0, 160), rng.integers(0, 4)
        Xp = X.copy(); Xp[i, j] += h
        Xm = X.copy(); Xm[i, j] -= h
        fd = (gcn.subspace_loss(Xp, U)[0] - gcn.subspace_loss(Xm, U)[0]) / (2 * h)
        assert abs(fd - dX[i, j]) <= 1e-7 * max(1.0, abs(fd))


def test_loss_gradient_fewer_targets_than_columns(small):
    """Targets narrower than the output block (the planted-cluster eigenvectors
    only): the loss and its gradient keep their definitions with k = ku."""
    gcn, csr, dims, W, X0, U = small
    X = np.random.default_rng(8).standard_normal((160, 4))
    U2 = U[:, :2]
    L, dX = gcn.subspace_loss(X, U2)
    assert 0.0 <= L <= 1.0
    h = 1e-6
    rng = np.random.default_rng(9)
    for _ in range(12):
        i, j = rng.integers(0, 160), rng.integers(0, 4)
        Xp = X.copy(); Xp[i, j] += h
        Xm = X.copy(); Xm[i, j] -= h
        fd = (gcn.subspace_loss(Xp, U2)[0] - gcn.subspace_loss(Xm, U2)[0]) / (2 * h)
        assert abs(fd - dX[i, j]) <= 1e-7 * max(1.0, abs(fd))
    # a block that contains the targets has loss 0 whatever its other columns
    Xc = np.concatenate([U2 @ np.array([[1.0, 2.0], [0.5, -1.0]]), X[:, :2]], 1)
    assert abs(gcn.subspace_loss(Xc, U2)[0]) < 1e-12


def test_weight_gradients_finite_differences(small):
    gcn, csr, dims, W, X0, U = small
    out, acts = gcn.forward(csr, X0, W)
    _, dX = gcn.subspace_loss(out, U)
    dW = gcn.backward(csr, X0, W, acts, dX)
    h = 1e-6
    rng = np.random.default_rng(7)
    for l in range(3):
        for _ in range(6):
            i, j = rng.integers(0, dims[l]), rng.integers(0, dims[l + 1])
            Wp = [w.copy() for w in W]; Wp[l][i, j] += h
            Wm = [w.copy() for w in W]; Wm[l][i, j] -= h
            fd = (_total_loss(gcn, csr, X0, Wp, U) - _total_loss(gcn, csr, X0, Wm, U)) / (2 * h)
            assert abs(fd - dW[l][i, j]) <= 1e-6 * max(1.0, abs(fd)), (l, i, j, fd, dW[l][i, j])


def test_loss_invariances_and_range(small):
    gcn, csr, dims, W, X0, U = small
    rng = np.random.default_rng(8)
    X = rng.standard_normal((160, 4))
    L = gcn.subspace_loss(X, U)[0]
    R = rng.standard_normal((4, 4)) + 4 * np.eye(4)          # invertible mixing of X
    assert abs(gcn.subspace_loss(X @ R, U)[0] - L) < 1e-12
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))         # rotation / signs of U
    assert abs(gcn.subspace_loss(X, U @ Q)[0] - L) < 1e-12
    assert 0.0 <= L <= 1.0
    assert abs(gcn.subspace_loss(U @ R, U)[0]) < 1e-12       # span(X) = span(U)
    Uc = np.linalg.qr(np.concatenate([U, X], 1))[0][:, 4:]   # complement of span(U)
    assert abs(gcn.subspace_loss(Uc, U)[0] - 1.0) < 1e-12
