"""Oracle (test infrastructure): Lanczos estimate of the spectrum bounds of A.

Sec. 2 notes that when the filter's bounds are unknown they can be estimated
by a few Lanczos steps.  Here: plain Lanczos (no reorthogonalization) from a
Philox start vector, then the Ritz values of the k x k tridiagonal T_k and the
bounds of Zhou & Li (2011): upper = max Ritz value + |beta_k|, lower = min Ritz
value - |beta_k|, where beta_k is the norm of the last residual vector.

Readings: the start vector is Philox column 2^32 - 1 of the seed (the column
number the solver's random vectors never reach), scaled to unit length; the
recurrence stops early when beta_j <= 1e-12 * max(1, |alpha_j|) (an invariant
subspace), and then beta_k is that last beta.  Each step is
    w = A v_j - beta_{j-1} v_{j-1};  alpha_j = v_j . w;  w = w - alpha_j v_j;
    beta_j = ||w||;  v_{j+1} = w / beta_j.
"""

from __future__ import annotations

import numpy as np

from ._lib import apply_laplacian
from .philox import random_block

START_COLUMN = 0xFFFFFFFF


def lanczos_bounds(csr, steps: int, seed: int):
    """Returns (lower, upper, alpha, beta)."""
    n = len(csr.deg)
    v = random_block(seed, n, [START_COLUMN])[:, 0].copy()
    v /= np.linalg.norm(v)
    v_prev = np.zeros(n)
    b_prev = 0.0
    alpha, beta = [], []
    for _ in range(steps):
        w = apply_laplacian(csr, np.asfortranarray(v[:, None]))[:, 0] - b_prev * v_prev
        a = float(v @ w)
        w = w - a * v
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b <= 1e-12 * max(1.0, abs(a)):
            break
        v_prev, v, b_prev = v, w / b, b
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    theta = np.linalg.eigvalsh(T)
    return float(theta[0] - beta[-1]), float(theta[-1] + beta[-1]), np.array(alpha), np.array(beta)
