"""Oracle: orthonormalization of a new block against the basis (Alg. 2, step 6).

Sec. 2 names DGKS (Daniel, Gragg, Kaufman & Stewart 1976): classical
Gram-Schmidt column by column, with one reorthogonalization when the norm drops
sharply, and replacement of numerically dependent vectors by random ones.  The
steps below follow that description, one column at a time, against
[V, accepted new columns]:

  1. nrm0 = ||x||;  x -= Q (Q^T x);  if ||x|| < eta nrm_before: x -= Q (Q^T x)
     again (eta = 1/sqrt(2), the classical DGKS constant);
  2. dependence (the paper gives no threshold; reading): the final norm is
     below tau_dep * nrm0 with tau_dep = 1e-10 (or nrm0 = 0).  A dependent column
     is replaced by the next Philox column and redone (at most 3 times);
  3. normalize.

Returns the orthonormal block, the number of replacements and the next free
random-column number.
"""

from __future__ import annotations

import numpy as np

from .philox import random_block

ETA = 1.0 / np.sqrt(2.0)
TAU_DEP = 1e-10
MAX_REPLACE = 3


def dgks(V: np.ndarray, X: np.ndarray, seed: int, next_col: int):
    """Orthonormalize the columns of X (n x kb) against V (n x ksub, orthonormal
    columns) and against each other."""
    n, kb = X.shape
    ksub = 0 if V is None else V.shape[1]
    Q = np.empty((n, ksub + kb), dtype=np.float64, order="F")
    if ksub:
        Q[:, :ksub] = V
    n_replaced = 0
    for j in range(kb):
        x = np.array(X[:, j], dtype=np.float64)
        tries = 0
        while True:
            basis = Q[:, : ksub + j]
            nrm0 = np.linalg.norm(x)
            nrm = nrm0
            if basis.shape[1]:
                for _ in range(2):
                    before = nrm
                    x = x - basis @ (basis.T @ x)
                    nrm = np.linalg.norm(x)
                    if nrm >= ETA * before:
                        break
            if nrm0 > 0.0 and nrm >= TAU_DEP * nrm0:
                break
            if tries == MAX_REPLACE:
                raise FloatingPointError("could not find an independent random vector")
            x = random_block(seed, n, [next_col])[:, 0]
            next_col += 1
            n_replaced += 1
            tries += 1
        Q[:, ksub + j] = x / nrm
    return np.asfortranarray(Q[:, ksub:]), n_replaced, next_col
