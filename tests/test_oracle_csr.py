"""Pins for the oracle's Laplacian construction (Eq. 1): the CSR pattern against a
brute-force dense adjacency, and dinv against exact rational arithmetic."""

from fractions import Fraction
import math

import numpy as np
import pytest


def _brute_force_adjacency(edges, n):
    S = [[0] * n for _ in range(n)]
    for u, v in edges:
        if u != v:
            S[u][v] = 1
            S[v][u] = 1
    return S


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_csr_matches_brute_force(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = 150
    raw = rng.integers(0, n, size=(900, 2))
    # duplicates in both orientations and self-loops on purpose
    raw = np.concatenate([raw, raw[:100, ::-1], raw[100:150], np.stack([np.arange(10)] * 2, 1)])
    g = oracle_mod.build_csr(raw, n)
    S = _brute_force_adjacency(raw.tolist(), n)
    rp = [0]
    cols = []
    for i in range(n):
        row = [j for j in range(n) if S[i][j]]
        cols += row
        rp.append(len(cols))
    assert g.row_ptr.tolist() == rp
    assert g.col.tolist() == cols
    assert g.deg.tolist() == [rp[i + 1] - rp[i] for i in range(n)]
    assert g.row_ptr.dtype == np.int64 and g.col.dtype == np.int32 and g.deg.dtype == np.int32


def test_isolated_nodes_and_rejects(oracle_mod):
    g = oracle_mod.build_csr(np.array([[0, 1], [1, 1]]), 4)
    assert g.deg.tolist() == [1, 1, 0, 0]
    assert g.dinv[2] == 0.0 and g.dinv[3] == 0.0
    A = oracle_mod.dense_laplacian(g)
    assert A[2, 2] == 1.0 and A[3, 3] == 1.0
    with pytest.raises(ValueError):
        oracle_mod.build_csr(np.array([[0, 4]]), 4)
    with pytest.raises(ValueError):
        oracle_mod.build_csr(np.array([[-1, 2]]), 4)
    g0 = oracle_mod.build_csr(np.zeros((0, 2), dtype=np.int64), 3)
    assert g0.nnz == 0 and g0.row_ptr.tolist() == [0, 0, 0, 0]


def _ulp(x: float) -> Fraction:
    return Fraction(math.ulp(x))


def _is_rn_sqrt(d: int, s: float) -> bool:
    h = _ulp(s) / 2
    fs = Fraction(s)
    return (fs - h) ** 2 < d < (fs + h) ** 2


def _is_rn_recip(s: float, q: float) -> bool:
    # |q - 1/s| < ulp(q)/2  <=>  |q s - 1| < s ulp(q)/2
    return abs(Fraction(q) * Fraction(s) - 1) < Fraction(s) * _ulp(q) / 2


def test_dinv_is_two_correctly_rounded_ops(oracle_mod):
    """dinv_i = RN(1 / RN(sqrt(deg_i))), checked with exact rational arithmetic on
    a union of stars whose centres take every degree 1..1500 plus large ones."""
    rng = np.random.default_rng(1)
    degs = np.concatenate([np.arange(1, 1501), rng.integers(1501, 200_000, size=20),
                           [2 ** 17 + 1, 250_000]]).astype(np.int64)
    parts, off = [], 0
    centres = []
    for d in degs.tolist():
        parts.append(np.stack([np.full(d, off, np.int64), np.arange(off + 1, off + d + 1)], 1))
        centres.append(off)
        off += d + 1
    g = oracle_mod.build_csr(np.concatenate(parts), off)
    assert g.deg[centres].tolist() == degs.tolist()
    for d, q in zip(degs.tolist(), g.dinv[centres].tolist()):
        s = math.sqrt(float(d))
        assert _is_rn_sqrt(d, s), d
        assert _is_rn_recip(s, q), d
    leaves = np.setdiff1d(np.arange(off), centres)
    assert (g.dinv[leaves] == 1.0).all()
