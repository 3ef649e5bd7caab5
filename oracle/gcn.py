"""Oracle (test infrastructure): the warm-start network and its training loss in
plain FP64 NumPy, with gradients by hand-written backpropagation.

Network (not part of the paper; it feeds the initial vectors of Alg. 2):
    Z_l = Ahat (H_{l-1} W_l),  H_l = max(Z_l, 0) for l = 1, 2,  X = Z_3,
    Ahat = D^{-1/2} S D^{-1/2} = I - A  (A the normalized Laplacian, Eq. 1).
Loss (invariant to rotations and signs of the targets U, n x k orthonormal):
    L(X) = 1 - tr(U^T X (X^T X)^{-1} X^T U) / k.

Gradients (derived by hand, pinned by central finite differences in the tests):
    dL/dX = -(2/k) (U M^T G^{-1} - X G^{-1} M M^T G^{-1}),  G = X^T X, M = X^T U;
    with G_l = Ahat dZ_l:  dW_l = H_{l-1}^T G_l,  dH_{l-1} = G_l W_l^T,
    dZ_{l-1} = dH_{l-1} * [H_{l-1} > 0].
"""

from __future__ import annotations

import numpy as np

from ._lib import apply_laplacian


def ahat(csr, X: np.ndarray) -> np.ndarray:
    """D^{-1/2} S D^{-1/2} X = X - A X."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    return X - apply_laplacian(csr, X)


def forward(csr, X0: np.ndarray, W):
    """Returns (out, [H1, H2])."""
    H = np.asarray(X0, dtype=np.float64)
    acts = []
    for l in range(3):
        Z = ahat(csr, H @ W[l])
        if l < 2:
            H = np.maximum(Z, 0.0)
            acts.append(H)
        else:
            out = Z
    return out, acts


def backward(csr, X0: np.ndarray, W, acts, d_out: np.ndarray):
    """Gradients of sum(out * d_out) with respect to W_1..W_3."""
    H = [np.asarray(X0, dtype=np.float64), acts[0], acts[1]]
    dW = [None, None, None]
    dZ = np.asarray(d_out, dtype=np.float64)
    for l in (2, 1, 0):
        G = ahat(csr, dZ)
        dW[l] = H[l].T @ G
        if l > 0:
            dH = G @ W[l].T
            dZ = dH * (H[l] > 0.0)
    return dW


def subspace_loss(X: np.ndarray, U: np.ndarray):
    """(L, dL/dX)."""
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    k = U.shape[1]
    G = X.T @ X
    M = X.T @ U
    Gi = np.linalg.inv(G)
    L = 1.0 - np.trace(M.T @ Gi @ M) / k
    dX = -(2.0 / k) * (U @ M.T @ Gi - X @ Gi @ M @ M.T @ Gi)
    return float(L), dX


def glorot(seed: int, dims):
    """Glorot-uniform weights for widths dims[0] -> dims[1] -> dims[2] -> dims[3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = []
    for l in range(3):
        a = np.sqrt(6.0 / (dims[l] + dims[l + 1]))
        W.append(rng.uniform(-a, a, size=(dims[l], dims[l + 1])))
    return W
