"""GPU: the Lanczos bound estimator (chebdav_lanczos_bounds) against the
oracle's restatement from the same Philox start vector, the interval against
the exact spectrum, and a solve with the estimated upper bound against the
oracle's solve with the same bound.

Tolerances: alpha_j and beta_j agree to 1e-11 (FP64 on both sides; the
recurrences differ only in summation order and the loss of orthogonality of
plain Lanczos amplifies that slowly over 20 steps); the bounds to 1e-10."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("steps", [1, 5, 20])
def test_matches_oracle(cd, oracle_mod, dev, steps):
    from oracle import lanczos
    e, n, _ = synth.make_config_graph("sbm5k")
    g = cd.build_laplacian(e, n)
    o = oracle_mod.build_csr(e, n)
    lo, hi, a, b = cd.lanczos_bounds(g, steps, seed=4)
    wlo, whi, wa, wb = lanczos.lanczos_bounds(o, steps, seed=4)
    print("steps %d: gpu [%.12f, %.12f] oracle [%.12f, %.12f]" % (steps, lo, hi, wlo, whi))
    assert len(a) == len(wa)
    assert np.abs(a - wa).max() <= 1e-11
    assert np.abs(b - wb).max() <= 1e-11
    assert abs(hi - whi) <= 1e-10 and abs(lo - wlo) <= 1e-10


def test_interval_contains_spectrum_and_early_stop(cd, oracle_mod, dev):
    e, n, _ = synth.make_config_graph("sbm5k")
    g = cd.build_laplacian(e, n)
    lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(oracle_mod.build_csr(e, n)))
    lo, hi, a, b = cd.lanczos_bounds(g, 12, seed=1)
    assert lo <= lam[0] + 1e-12 and hi >= lam[-1] - 1e-12
    print("sbm5k: lambda_max %.6f, estimated upper bound %.6f" % (lam[-1], hi))
    # complete graph K_8: an invariant subspace after two steps, exact extremes
    g8 = cd.build_laplacian(synth.complete_graph(8), 8)
    lo, hi, a, b = cd.lanczos_bounds(g8, 10, seed=3)
    assert len(a) == 2 and abs(hi - 8.0 / 7.0) <= 1e-11


def test_errors(cd, dev):
    g = cd.build_laplacian(synth.cycle_graph(10), 10)
    with pytest.raises(cd.ChebdavError):
        cd.lanczos_bounds(g, 0)
    with pytest.raises(cd.ChebdavError):
        cd.lanczos_bounds(g, 257)


def test_solve_with_estimated_upper_bound(cd, oracle_mod, dev):
    """Alg. 2 with b from the estimator instead of the analytic 2: same
    eigenpairs as the oracle run with that b, and no more iterations than b = 2."""
    e, n, cfg = synth.make_config_graph("sbm5k")
    g = cd.build_laplacian(e, n)
    o = oracle_mod.build_csr(e, n)
    _, hi, _, _ = cd.lanczos_bounds(g, 10, seed=1)
    ub = min(hi, 2.0)
    p = cd.make_params(k_want=4, kb=4, m=11, seed=1, upperb=ub)
    r = cd.solve(g, p)
    r2 = cd.solve(g, cd.make_params(k_want=4, kb=4, m=11, seed=1))
    ref = oracle_mod.bchdav(o, oracle_mod.Params(k_want=4, kb=4, m=11, seed=1, upperb=ub))
    ev, V = r.evals.cpu().numpy(), r.evecs.cpu().numpy()
    R = oracle_mod.apply_laplacian(o, np.asfortranarray(V)) - V * ev
    print("upper bound %.6f: %d iterations (oracle %d); b = 2: %d iterations"
          % (ub, r.stats["iterations"], ref.iterations, r2.stats["iterations"]))
    assert np.sqrt((R * R).sum(0)).max() <= 1e-8
    assert np.abs(ev - ref.evals).max() <= 1e-10
    assert abs(r.stats["iterations"] - ref.iterations) <= 2
