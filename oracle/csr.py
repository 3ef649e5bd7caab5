"""Oracle: the canonical CSR pattern of S and the degree scaling of Eq. 1.

Definition (Eq. 1): S_ij = 1 iff nodes i and j are connected, so the graph is
simple.  Reading of the undefined cases: self-loops are dropped, repeated
edges (in either orientation) are merged, and an isolated node has
dinv = 0, which makes its row of A the identity row (eigenvalue 1).

CSR layout: row_ptr int64[n+1], col int32[nnz] ascending within each row,
deg int32[n] = row lengths, dinv float64[n] = 1.0 / sqrt(deg) with IEEE
round-to-nearest sqrt and division (0 where deg = 0).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    deg: np.ndarray
    dinv: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def build_csr(edges, n: int) -> CSR:
    """Canonical symmetric CSR of the simple graph given by an edge list."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if n <= 0:
        raise ValueError("n must be positive")
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("node id outside [0, n)")
    e = e[e[:, 0] != e[:, 1]]
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    key = np.unique(rows * np.int64(n) + cols)          # sorted, duplicates merged
    r = key // n
    c = key - r * n
    counts = np.bincount(r, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    deg = counts.astype(np.int32)
    dinv = np.zeros(n, dtype=np.float64)
    nz = deg > 0
    dinv[nz] = 1.0 / np.sqrt(deg[nz].astype(np.float64))
    return CSR(n=n, row_ptr=row_ptr, col=c.astype(np.int32), deg=deg, dinv=dinv)


def dense_laplacian(csr: CSR) -> np.ndarray:
    """Dense A = I - D^{-1/2} S D^{-1/2} (small n only)."""
    n = csr.n
    S = np.zeros((n, n))
    r = np.repeat(np.arange(n), np.diff(csr.row_ptr))
    S[r, csr.col] = 1.0
    return np.eye(n) - csr.dinv[:, None] * S * csr.dinv[None, :]
