"""Pins for the oracle's Chebyshev filter (Alg. 3) against the closed form of
Eqs. 3-5: p_m(A) X = Q p_m(Lambda) Q^T X with
p_m(x) = C_m(ell(x)) / C_m(ell(a0)), ell(x) = (x - c)/e, and C_m evaluated from
its trigonometric / hyperbolic definition (Eq. 4), never from the recurrence."""

import math

import numpy as np
import pytest

import synth


def cheb_closed(mdeg, x):
    """C_m(x) by Eq. 4."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(mdeg * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** mdeg * np.cosh(mdeg * np.arccosh(np.abs(xo)))
    return out


def p_m(mdeg, lam, cut, upper, a0):
    c = (upper + cut) / 2
    e = (upper - cut) / 2
    return cheb_closed(mdeg, (lam - c) / e) / cheb_closed(mdeg, np.array([(a0 - c) / e]))[0]


@pytest.mark.parametrize("mdeg,cut", [(1, 0.3), (2, 0.5), (11, 0.2), (15, 0.6), (20, 0.05)])
def test_filter_closed_form_dense(oracle_mod, mdeg, cut):
    e, _ = synth.sbm(300, 3, p_in=0.1, p_out=0.01, seed=mdeg)
    g = oracle_mod.build_csr(e, 300)
    A = oracle_mod.dense_laplacian(g)
    lam, Q = np.linalg.eigh(A)
    X = np.random.default_rng(mdeg).standard_normal((300, 5))
    want = Q @ (p_m(mdeg, lam, cut, 2.0, 0.0)[:, None] * (Q.T @ X))
    got = oracle_mod.cheb_filter(g, X, mdeg, cut, 2.0, 0.0)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-11 * scale


def test_filter_bounded_on_damped_interval(oracle_mod):
    lam = np.linspace(0.3, 2.0, 1001)
    assert np.abs(p_m(20, lam, 0.3, 2.0, 0.0)).max() <= 1.0 / cheb_closed(20, np.array([-(2.3 / 1.7)]))[0] * 1.0000001
    assert p_m(20, np.array([0.0]), 0.3, 2.0, 0.0)[0] == pytest.approx(1.0, rel=1e-14)


def test_sigma_schedule_closed_form(oracle_mod):
    cut, upper, a0 = 0.4, 2.0, 0.0
    c, e, sig = oracle_mod.sigma_schedule(12, cut, upper, a0)
    l0 = np.array([(a0 - c) / e])
    for k in range(1, 13):
        want = cheb_closed(k - 1, l0)[0] / cheb_closed(k, l0)[0]
        assert sig[k - 1] == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("n,j,mdeg,cut", [(100_000, 3, 15, 0.2), (65_536, 1000, 11, 0.01), (7, 2, 20, 0.5)])
def test_filter_cycle_fourier_modes(oracle_mod, n, j, mdeg, cut):
    """On the cycle C_n, cos(2 pi j x / n) is an eigenvector with eigenvalue
    1 - cos(2 pi j / n), so the filter must return p_m(lambda_j) times it."""
    g = oracle_mod.build_csr(synth.cycle_graph(n), n)
    ph = 2 * math.pi * ((j * np.arange(n, dtype=np.int64)) % n) / n   # exact phase reduction
    X = np.stack([np.cos(ph), np.sin(ph)], 1)
    lam = 1 - math.cos(2 * math.pi * j / n)
    got = oracle_mod.cheb_filter(g, X, mdeg, cut, 2.0, 0.0)
    f = p_m(mdeg, np.array([lam]), cut, 2.0, 0.0)[0]
    assert np.abs(got - f * X).max() <= 1e-12 * max(1.0, abs(f))


def test_filter_rejects_bad_interval(oracle_mod):
    g = oracle_mod.build_csr(synth.cycle_graph(10), 10)
    with pytest.raises(ValueError):
        oracle_mod.cheb_filter(g, np.ones((10, 1)), 3, 0.0, 2.0, 0.0)
    with pytest.raises(ValueError):
        oracle_mod.cheb_filter(g, np.ones((10, 1)), 0, 0.5, 2.0, 0.0)


def test_apply_matches_dense(oracle_mod):
    e, _ = synth.sbm(400, 4, p_in=0.08, p_out=0.005, seed=2)
    e = np.concatenate([e, [[5, 5]], e[:20, ::-1]])
    g = oracle_mod.build_csr(e, 402)   # two isolated nodes
    A = oracle_mod.dense_laplacian(g)
    X = np.random.default_rng(0).standard_normal((402, 7))
    for Xo in (X, np.asfortranarray(X)):
        Y = oracle_mod.apply_laplacian(g, Xo)
        assert np.abs(Y - A @ X).max() < 1e-13
    # A is symmetric with spectrum in [0, 2]
    assert np.allclose(A, A.T)
    lam = np.linalg.eigvalsh(A)
    assert lam.min() > -1e-12 and lam.max() < 2 + 1e-12
