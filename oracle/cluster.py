"""Oracle (test infrastructure): the clustering tail of spectral clustering
(Alg. 1, steps 3 and 4) in plain FP64 NumPy, and the two agreement scores used
to score a partition against the planted blocks.

Readings (the paper names K-means and row normalization only):
  * a row is divided by its 2-norm (the plain definition; no summation order
    is implied); a zero row of the eigenvector block stays zero;
  * K-means is Lloyd's iteration (assign every row to its nearest centre by
    squared Euclidean distance, ties to the lower centre index; move every
    centre to the mean of its rows; a centre with no rows stays where it is),
    stopped when no assignment changes or after max_iter rounds;
  * initial centres by farthest-first traversal (Gonzalez, 1985): the first is
    row floor(u n) for the Philox4x32-10 draw u of counter (0, 0, 0, 1) under
    the seed (integer arithmetic), each next one the row with the largest distance to its nearest
    chosen centre (ties to the lower row index);
  * a squared distance is summed over the coordinates in ascending order, one
    rounded subtraction, product and sum each (no fused multiply-add).

Scores (pinned in the tests by brute-force pair counting and by exact cases):
  * adjusted Rand index (Hubert & Arabie, 1985) from the contingency table;
  * normalized mutual information I(a; b) / sqrt(H(a) H(b)) (Strehl & Ghosh, 2002).
"""

from __future__ import annotations

import numpy as np

from .philox import philox4x32_10


def row_normalize(U: np.ndarray) -> np.ndarray:
    """Each row divided by its 2-norm; zero rows stay zero."""
    U = np.asarray(U, dtype=np.float64)
    nr = np.sqrt((U * U).sum(axis=1))
    out = np.zeros_like(U)
    nz = nr > 0.0
    out[nz] = U[nz] / nr[nz, None]
    return out


def sq_dist(F: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Squared distances of every row of F to the point c, coordinates summed in
    ascending order without fused operations."""
    d = np.zeros(F.shape[0])
    for j in range(F.shape[1]):
        t = F[:, j] - c[j]
        d = d + t * t
    return d


def first_index(n: int, seed: int) -> int:
    """floor(u n) with u the 53-bit Philox4x32-10 draw of counter (0, 0, 0, 1)
    and key (seed mod 2^32, seed >> 32), in integer arithmetic."""
    w = philox4x32_10(0, 0, 0, 1, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u53 = ((int(w[1]) << 32) | int(w[0])) >> 11
    return (u53 * n) >> 53


def farthest_first(F: np.ndarray, K: int, seed: int) -> np.ndarray:
    """Indices of the K initial centres."""
    n = F.shape[0]
    idx = [first_index(n, seed)]
    mind = sq_dist(F, F[idx[0]])
    for _ in range(1, K):
        i = int(np.argmax(mind))  # first maximum = lowest index among ties
        idx.append(i)
        mind = np.minimum(mind, sq_dist(F, F[i]))
    return np.array(idx, dtype=np.int64)


def kmeans(F: np.ndarray, K: int, seed: int = 0, max_iter: int = 100):
    """Lloyd's K-means from farthest-first centres.
    Returns (labels int32[n], centres K x k, rounds, inertia), where rounds counts
    the assignment passes and inertia is the sum of squared distances of the
    final assignment."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    C = F[farthest_first(F, K, seed)].copy()
    labels = np.full(n, -1, dtype=np.int32)
    rounds = 0
    while rounds < max_iter:
        rounds += 1
        D = np.stack([sq_dist(F, C[c]) for c in range(K)], axis=1)
        new = np.argmin(D, axis=1).astype(np.int32)  # first minimum = lower centre index
        changed = int((new != labels).sum())
        labels = new
        for c in range(K):
            members = labels == c
            if members.any():
                C[c] = F[members].sum(axis=0) / members.sum()
        if changed == 0:
            break
    D = np.stack([sq_dist(F, C[c]) for c in range(K)], axis=1)
    inertia = float(D[np.arange(n), labels].sum())
    return labels, C, rounds, inertia


def contingency(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    M = np.zeros((ai.max() + 1, bi.max() + 1), dtype=np.int64)
    np.add.at(M, (ai, bi), 1)
    return M


def _comb2(x):
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) / 2.0


def ari(a, b) -> float:
    """Adjusted Rand index: (sum_ij C(n_ij,2) - E) / (max - E) with
    E = sum_i C(a_i,2) sum_j C(b_j,2) / C(n,2), max = (sum_i C(a_i,2) + sum_j C(b_j,2)) / 2."""
    M = contingency(a, b)
    n = M.sum()
    sij = _comb2(M).sum()
    sa = _comb2(M.sum(axis=1)).sum()
    sb = _comb2(M.sum(axis=0)).sum()
    e = sa * sb / _comb2(n)
    mx = 0.5 * (sa + sb)
    if mx == e:
        return 1.0
    return float((sij - e) / (mx - e))


def nmi(a, b) -> float:
    """I(a; b) / sqrt(H(a) H(b)), natural logarithms; 1 when both are single clusters."""
    M = contingency(a, b).astype(np.float64)
    n = M.sum()
    pa = M.sum(axis=1) / n
    pb = M.sum(axis=0) / n
    ha = -float(np.sum(pa * np.log(pa)))
    hb = -float(np.sum(pb * np.log(pb)))
    nz = M > 0
    pij = M[nz] / n
    outer = np.outer(pa, pb)[nz]
    mi = float(np.sum(pij * np.log(pij / outer)))
    if ha == 0.0 or hb == 0.0:
        return 1.0 if ha == hb else 0.0
    return mi / np.sqrt(ha * hb)
