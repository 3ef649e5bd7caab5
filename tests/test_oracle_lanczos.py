"""Pins for the oracle's Lanczos bound estimator (Sec. 2): Ritz values of a
symmetric matrix lie inside its spectrum, the estimated interval contains the
whole spectrum of the test graphs (dense eigh), and on a small matrix the full
Lanczos run reproduces the spectrum."""

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def lz(oracle_mod):
    from oracle import lanczos
    return lanczos


@pytest.mark.parametrize("name", ["sbm", "cycle_odd", "path", "complete", "star"])
def test_bounds_contain_spectrum(oracle_mod, lz, name):
    if name == "sbm":
        e, _ = synth.sbm(600, 4, p_in=0.05, p_out=0.004, seed=2)
        n = 600
    elif name == "cycle_odd":
        e, n = synth.cycle_graph(301), 301
    elif name == "path":
        e, n = synth.path_graph(200), 200
    elif name == "complete":
        e, n = synth.complete_graph(40), 40
    else:
        e, n = synth.star_graph(50), 50
    g = oracle_mod.build_csr(e, n)
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(g))
    for steps in (6, 12, 20):
        lo, hi, a, b = lz.lanczos_bounds(g, steps, seed=7)
        T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
        theta = np.linalg.eigvalsh(T)
        # Ritz values of a symmetric matrix lie in [lambda_min, lambda_max]
        assert theta[0] >= lam[0] - 1e-10 and theta[-1] <= lam[-1] + 1e-10
        assert hi >= lam[-1] - 1e-10, (name, steps, hi, lam[-1])
        assert lo <= lam[0] + 1e-10


def test_full_run_reproduces_spectrum(oracle_mod, lz):
    # complete graph K_8: eigenvalues 0 and 8/7 (x7); Lanczos ends at an invariant
    # subspace after two steps, with the extreme eigenvalues as Ritz values
    e, n = synth.complete_graph(8), 8
    g = oracle_mod.build_csr(e, n)
    lo, hi, a, b = lz.lanczos_bounds(g, 10, seed=3)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    theta = np.linalg.eigvalsh(T)
    assert len(a) == 2
    assert abs(theta[0]) < 1e-13 and abs(theta[-1] - 8.0 / 7.0) < 1e-13
    assert abs(hi - 8.0 / 7.0) < 1e-11
