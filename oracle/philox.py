"""Oracle: the counter-based generator the solver draws its random vectors from.

The paper fills missing start vectors (Alg. 2, step 2) and replaces
numerically dependent vectors (Sec. 2, orthonormalization) with "random
vectors" without fixing a distribution.  Reading: Philox4x32-10 (Salmon, Moraes,
Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), written
here from that published definition:

  * state: counter (c0, c1, c2, c3) and key (k0, k1), 32-bit words;
  * one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
    new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
    with M0 = 0xD2511F53, M1 = 0xCD9E8D57;
  * ten rounds; between rounds the key is bumped by the Weyl constants
    (0x9E3779B9, 0xBB67AE85).

Entry (row r, random column number q) of a random block uses
counter = (r mod 2^32, r >> 32, q, 0), key = (seed mod 2^32, seed >> 32), and the
first two output words w0, w1 form u = ((w1 << 32) | w0) >> 11, a 53-bit integer;
the value is u * 2^-52 - 1, which is exact and uniform on [-1, 1).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorized Philox4x32-10 over arrays of uint32 counters; returns 4 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = np.uint32(k0 + W0)
                k1 = np.uint32(k1 + W1)
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def random_block(seed: int, n: int, col_ids) -> np.ndarray:
    """n x len(col_ids) block of uniform [-1, 1) values (column-major)."""
    col_ids = np.asarray(col_ids, dtype=np.uint64).reshape(-1)
    rows = np.arange(n, dtype=np.uint64)
    out = np.empty((n, col_ids.size), dtype=np.float64, order="F")
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    r_lo = (rows & _MASK32).astype(np.uint32)
    r_hi = (rows >> np.uint64(32)).astype(np.uint32)
    zero = np.zeros(n, dtype=np.uint32)
    for t, q in enumerate(col_ids):
        qv = np.full(n, np.uint32(int(q) & 0xFFFFFFFF), dtype=np.uint32)
        w0, w1, _, _ = philox4x32_10(r_lo, r_hi, qv, zero, k0, k1)
        u = ((w1.astype(np.uint64) << np.uint64(32)) | w0.astype(np.uint64)) >> np.uint64(11)
        out[:, t] = u.astype(np.float64) * 2.0 ** -52 - 1.0
    return out
