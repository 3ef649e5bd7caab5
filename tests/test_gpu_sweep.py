"""GPU: a seeded sweep over solver configurations — SBM and Chung-Lu graphs of
300 to 40k nodes, block sizes 1 to 32 (odd ones included), k from 1 to 3 kb + 1,
filter degrees 5 to 20, FP64 and FP32-filter forms, tolerances 1e-6 to 1e-10,
Cholesky-QR and TSQR orthonormalization.  Every solve must return OK with
every fresh residual, computed by the oracle's own sparse product, within its
tolerance and an orthonormal basis; on graphs up to 1500 nodes the eigenvalues
are also compared with dense LAPACK eigh: each of the k Ritz values lies
within its residual of an eigenvalue (Weinstein's bound), so matching the k
smallest in order to within tol shows that none was missed."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _case(rng):
    kind = rng.choice(["sbm", "cl", "sbm_small"])
    if kind == "sbm":
        n = int(rng.integers(3000, 30000))
        e, _ = synth.sbm(n, int(rng.integers(2, 40)), d_in=float(rng.uniform(8, 25)),
                         d_out=float(rng.uniform(1, 5)), uneven=True, seed=int(rng.integers(1 << 30)))
    elif kind == "cl":
        e, n = synth.chung_lu(int(rng.integers(5000, 40000)), seed=int(rng.integers(1 << 30)))
    else:
        n = int(rng.integers(300, 1500))
        e, _ = synth.sbm(n, int(rng.integers(2, 10)), d_in=float(rng.uniform(6, 15)),
                         d_out=float(rng.uniform(0.5, 3)), uneven=True, seed=int(rng.integers(1 << 30)))
    kb = int(rng.choice([1, 2, 3, 4, 5, 7, 8, 12, 16, 24, 32]))
    k = int(max(1, min(rng.integers(1, 3 * kb + 2), 48)))
    return dict(kind=str(kind), e=e, n=n, kb=kb, k=k, m=int(rng.integers(5, 21)), f32=bool(rng.integers(0, 2)),
                seed=int(rng.integers(1 << 30)), tol=float(rng.choice([1e-6, 1e-8, 1e-8, 1e-10])),
                orth=str(rng.choice(["cholqr", "cholqr", "tsqr"])))


def test_configuration_sweep(cd, oracle_mod, dev):
    rng = np.random.default_rng(20240607)
    for i in range(24):
        c = _case(rng)
        print("case %d %s n=%d k=%d kb=%d m=%d %s tol=%.0e %s seed=%d" % (
            i, c["kind"], c["n"], c["k"], c["kb"], c["m"], "f32" if c["f32"] else "f64", c["tol"], c["orth"],
            c["seed"]), flush=True)
        g = cd.build_laplacian(c["e"], c["n"])
        p = cd.make_params(k_want=c["k"], kb=c["kb"], m=c["m"], seed=c["seed"], tol=c["tol"], itmax=400,
                           filter_dtype=cd.F32 if c["f32"] else cd.F64, orth=c["orth"])
        r = cd.solve(g, p)
        ev, V = r.evals.cpu().numpy(), r.evecs.cpu().numpy()
        o = oracle_mod.build_csr(c["e"], c["n"])
        R = oracle_mod.apply_laplacian(o, np.asfortranarray(V)) - V * ev
        res = np.sqrt((R * R).sum(0))
        assert res.max() <= c["tol"] * 1.01, res.max()
        assert np.linalg.norm(V.T @ V - np.eye(c["k"]), 2) <= 1e-10
        if c["n"] <= 1500:
            lam = np.linalg.eigvalsh(oracle_mod.dense_laplacian(o))
            assert np.abs(ev - lam[:c["k"]]).max() <= c["tol"]
