"""Oracle (test infrastructure): tall-skinny QR.

Sec. 3.3 orthonormalizes distributed blocks with the parallel TSQR of Demmel et
al.: every row block is factored on its own, the R factors of q neighbouring
blocks are stacked in block order and factored again, up a tree, until one R
is left; Q is the product of the block-diagonal intermediate Q factors.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.

householder_qr is the plain definition the GPU path is compared with: the thin
QR of X by Householder reflections, column by column, with the signs chosen so
that R has a non-negative diagonal (for X of full column rank that QR is
unique).  tsqr_tree restates the paper's tree (leaves = row blocks, fan-in q)
on top of it; the tests check that both give the same factors.

Reading: a reflector zeroes the entries below the diagonal of its column and
leaves a column that is already zero there untouched (as LAPACK's does).
"""

from __future__ import annotations

import numpy as np


def householder_qr(X):
    """Thin QR of X (n x k, n >= k): returns Q (n x k, orthonormal columns) and
    R (k x k, upper triangular, diagonal >= 0) with X = Q R."""
    A = np.array(X, dtype=np.float64, copy=True)
    n, k = A.shape
    if n < k:
        raise ValueError("householder_qr needs n >= k")
    vs, taus = [], []
    for j in range(k):
        x = A[j:, j]
        alpha = x[0]
        sub = float(np.dot(x[1:], x[1:]))
        if sub == 0.0:
            vs.append(None)
            taus.append(0.0)
            continue
        norm = np.sqrt(alpha * alpha + sub)
        beta = -norm if alpha >= 0 else norm
        v = x / (alpha - beta)
        v[0] = 1.0
        tau = (beta - alpha) / beta
        # apply H = I - tau v v^T to the remaining columns
        A[j:, j:] -= tau * np.outer(v, v @ A[j:, j:])
        A[j + 1:, j] = 0.0
        A[j, j] = beta
        vs.append(v)
        taus.append(tau)
    R = np.triu(A[:k, :])
    # Q = H_0 H_1 ... H_{k-1} [I; 0]
    Q = np.zeros((n, k))
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        if vs[j] is None:
            continue
        v = vs[j]
        Q[j:, :] -= taus[j] * np.outer(v, v @ Q[j:, :])
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def tsqr_tree(X, p: int, q: int):
    """The paper's parallel TSQR with p leaves (row blocks of nearly equal size,
    in order) and fan-in q, executed sequentially.  Returns (Q, R)."""
    X = np.asarray(X, dtype=np.float64)
    n, k = X.shape
    bounds = np.linspace(0, n, p + 1).astype(int)
    blocks = [X[bounds[i]:bounds[i + 1]] for i in range(p)]
    if any(b.shape[0] < k for b in blocks):
        raise ValueError("every leaf needs at least k rows")
    # level 0: local QR of every row block
    Qs = []   # Qs[level][i]: Q factor of node i at that level
    Rs = []
    level_q, level_r = zip(*(householder_qr(b) for b in blocks))
    Qs.append(list(level_q))
    Rs = list(level_r)
    while len(Rs) > 1:
        nq, nr = [], []
        for i in range(0, len(Rs), q):
            C = np.vstack(Rs[i:i + q])   # stacked R factors in node order
            Qc, Rc = householder_qr(C)
            nq.append(Qc)
            nr.append(Rc)
        Qs.append(nq)
        Rs = nr
    # Q = diag(Q_{.,0}) diag(Q_{.,1}) ... Q_{top}, evaluated top-down
    Y = Qs[-1][0]
    for level in range(len(Qs) - 2, -1, -1):
        parts = []
        for i, Qi in enumerate(Qs[level]):
            parts.append(Qi @ Y[i * k:(i + 1) * k])
        Y = np.vstack(parts)
    return Y, Rs[0]
