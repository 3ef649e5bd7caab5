"""Oracle: the scaled Chebyshev filter of Alg. 3 (Sec. 2, Eqs. 3-5).

Readings of the garbled passages:
  * roles of the three interval ends: `cut` is the lower end of the unwanted
    interval (updated to the median of the non-converged Ritz values, Alg. 2
    step 18), `upper` = b = 2 is the spectrum's upper bound, and `scale_pt` = a0
    = 0 is its lower bound, where the filter is normalized to 1.  Only this
    assignment damps [cut, upper] and amplifies [scale_pt, cut), which is what
    Sec. 2 says the filter is for;
  * the fixed constant of the sigma update is tau = 2 / sigma_1 (the printed
    "t" and "tau" are the same symbol), and the lowercase "v" in the update is
    the block from the previous degree.

With ell(x) = (x - c)/e, c = (cut + upper)/2, e = (upper - cut)/2, the steps
compute U_k = C_k(ell(A)) X / C_k(ell(scale_pt)) for k = 1..m, so the result is
p_m(A) X with p_m(x) = C_m(ell(x)) / C_m(ell(scale_pt)) (Eqs. 3-5).
"""

from __future__ import annotations

import numpy as np

from ._lib import apply_laplacian


def sigma_schedule(m: int, cut: float, upper: float, scale_pt: float):
    """(c, e, [sigma_1, ..., sigma_m]) as Alg. 3 produces them."""
    e = (upper - cut) / 2.0
    c = (upper + cut) / 2.0
    sigma = e / (scale_pt - c)
    tau = 2.0 / sigma
    sig = [sigma]
    for _ in range(2, m + 1):
        sigma = 1.0 / (tau - sigma)
        sig.append(sigma)
    return c, e, sig


def cheb_filter(csr, X: np.ndarray, m: int, cut: float, upper: float = 2.0,
                scale_pt: float = 0.0) -> np.ndarray:
    """Y = p_m(A) X by the three-term recurrence of Alg. 3, in FP64."""
    if m < 1:
        raise ValueError("m >= 1")
    if not (scale_pt < cut < upper):
        raise ValueError("need scale_pt < cut < upper")
    X = np.asarray(X, dtype=np.float64)
    e = (upper - cut) / 2.0
    c = (upper + cut) / 2.0
    sigma = e / (scale_pt - c)
    tau = 2.0 / sigma
    prev = X
    cur = (apply_laplacian(csr, X) - c * X) * (sigma / e)
    for _ in range(2, m + 1):
        sigma1 = 1.0 / (tau - sigma)
        nxt = (2.0 * sigma1 / e) * (apply_laplacian(csr, cur) - c * cur) - (sigma * sigma1) * prev
        prev, cur, sigma = cur, nxt, sigma1
    return cur
