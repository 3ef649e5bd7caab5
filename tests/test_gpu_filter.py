"""GPU parity: the fused sparse step and the Chebyshev filter (Alg. 3) against
the oracle (FP64, and the FP32 form), plus cycle-graph Fourier modes at scale.

Tolerances (max abs error / max abs value of the result):
  * sparse step FP64: 1e-14.  Each output is x_i - d_i sum_j d_j x_j over at
    most a few dozen terms, so rounding differs from the oracle's (which takes
    no fused multiply-add) by a few ulps of the largest term.
  * filter FP64: 1e-12.  Every degree applies one such step to a block that
    stays bounded (|p_k| <= 1 on the spectrum), so the errors add up over m <= 20
    steps with growth bounded by the Chebyshev recurrence (about 2 per step
    relative to the block scale in the worst case).
  * FP32 sparse step: 2e-6 (a few FP32 ulps, 6e-8 each, times the row sum).
  * FP32 filter: 1e-4 (the FP64 argument with eps = 6e-8).
"""

import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _rel_err(got, want):
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


@pytest.fixture(scope="module")
def sbm20k(cd, oracle_mod, dev):
    e, _ = synth.sbm(20_003, 16, d_in=20, d_out=4, uneven=True, seed=5)
    e = np.concatenate([e, [[7, 7]]])   # a self-loop; nodes 20001, 20002 may be isolated
    n = 20_005
    return cd.build_laplacian(e, n), oracle_mod.build_csr(e, n)


@pytest.mark.parametrize("kb,pad", [(1, 0), (4, 0), (5, 3), (30, 2), (32, 0), (64, 0), (130, 6)])
def test_spmm_f64_matches_oracle(cd, oracle_mod, sbm20k, kb, pad):
    import torch
    g, o = sbm20k
    rng = np.random.default_rng(kb)
    U = rng.standard_normal((o.n, kb + pad))
    Z = rng.standard_normal((o.n, kb + pad))
    Ut = torch.from_numpy(U).cuda()
    Zt = torch.from_numpy(Z).cuda()
    Yt = torch.full_like(Ut, 7.0)
    print("case spmm f64 kb=%d pad=%d" % (kb, pad), flush=True)
    cd.spmm(g, -1.0, 1.0, 0.0, Ut[:, :kb], None, Yt[:, :kb])
    Y = Yt.cpu().numpy()
    want = oracle_mod.apply_laplacian(o, np.ascontiguousarray(U[:, :kb]))
    assert _rel_err(Y[:, :kb], want) <= 1e-14
    assert (Y[:, kb:] == 7.0).all()                    # padding untouched
    # general coefficients: alpha (U - AU) + beta U + gamma Z
    a, b, c = 0.7, -1.3, 0.25
    cd.spmm(g, a, b, c, Ut[:, :kb], Zt[:, :kb], Yt[:, :kb])
    want2 = a * (U[:, :kb] - want) + b * U[:, :kb] + c * Z[:, :kb]
    assert _rel_err(Yt.cpu().numpy()[:, :kb], want2) <= 1e-14


@pytest.mark.parametrize("kb", [4, 32, 64])
def test_spmm_f32_matches_oracle(cd, oracle_mod, sbm20k, kb):
    import torch
    g, o = sbm20k
    U32 = np.random.default_rng(kb).standard_normal((o.n, kb)).astype(np.float32)
    Ut = torch.from_numpy(U32).cuda()
    Yt = torch.empty_like(Ut)
    print("case spmm f32 kb=%d" % kb, flush=True)
    cd.spmm(g, -1.0, 1.0, 0.0, Ut, None, Yt)
    want = oracle_mod.apply_laplacian(o, U32.astype(np.float64))
    assert _rel_err(Yt.cpu().numpy().astype(np.float64), want) <= 2e-6


@pytest.mark.parametrize("m,cut,kb", [(1, 0.3, 4), (2, 0.5, 5), (11, 0.05, 32), (15, 0.6, 64), (20, 0.2, 32)])
def test_filter_f64_matches_oracle(cd, oracle_mod, sbm20k, m, cut, kb):
    import torch
    g, o = sbm20k
    X = np.random.default_rng(m).standard_normal((o.n, kb))
    print("case filter f64 m=%d cut=%g kb=%d" % (m, cut, kb), flush=True)
    Y = cd.filter(g, torch.from_numpy(X).cuda(), m, cut, 2.0, 0.0).cpu().numpy()
    want = oracle_mod.cheb_filter(o, X, m, cut, 2.0, 0.0)
    assert _rel_err(Y, want) <= 1e-12


@pytest.mark.parametrize("m,cut,kb", [(11, 0.05, 4), (15, 0.6, 32), (20, 0.2, 64)])
def test_filter_f32_matches_oracle(cd, oracle_mod, sbm20k, m, cut, kb):
    import torch
    g, o = sbm20k
    X = np.random.default_rng(m).standard_normal((o.n, kb))
    print("case filter f32 m=%d" % m, flush=True)
    Y = cd.filter(g, torch.from_numpy(X).cuda(), m, cut, 2.0, 0.0, dtype=cd.F32).cpu().numpy()
    want = oracle_mod.cheb_filter(o, X, m, cut, 2.0, 0.0)
    err = _rel_err(Y, want)
    print("f32 filter rel err %.3g" % err)
    assert err <= 1e-4


def test_filter_strided_output(cd, oracle_mod, sbm20k):
    import torch
    g, o = sbm20k
    X = np.random.default_rng(1).standard_normal((o.n, 8))
    big = torch.zeros(o.n, 40, dtype=torch.float64, device="cuda")
    Xt = torch.zeros(o.n, 12, dtype=torch.float64, device="cuda")
    Xt[:, :8] = torch.from_numpy(X).cuda()
    cd.filter(g, Xt[:, :8], 9, 0.4, 2.0, 0.0, Y=big[:, 16:24])
    Y = big.cpu().numpy()
    assert _rel_err(Y[:, 16:24], oracle_mod.cheb_filter(o, X, 9, 0.4)) <= 1e-12
    assert (Y[:, :16] == 0).all() and (Y[:, 24:] == 0).all()


def _p_m(m, lam, cut, upper=2.0, a0=0.0):
    c, e = (upper + cut) / 2, (upper - cut) / 2

    def C(mm, x):
        return math.cos(mm * math.acos(x)) if abs(x) <= 1 else \
            math.copysign(1, x) ** mm * math.cosh(mm * math.acosh(abs(x)))
    return C(m, (lam - c) / e) / C(m, (a0 - c) / e)


@pytest.mark.parametrize("dt,tol", [(0, 1e-11), (1, 2e-4)])
def test_cycle_fourier_modes_at_scale(cd, dev, dt, tol):
    """C_n with n = 10^6: cos(2 pi j x/n) and sin(...) are eigenvectors with
    eigenvalue 1 - cos(2 pi j/n); the filter must scale them by p_m(lambda_j)."""
    import torch
    n = 1_000_000
    g = cd.build_laplacian(synth.cycle_graph(n), n)
    x = torch.arange(n, dtype=torch.int64, device=dev)
    js = [1, 17, 250_000, 400_000]
    # the phase j x mod n is reduced exactly in integers, so the sampled modes are
    # eigenvectors to rounding level
    X = torch.stack([f(2 * math.pi * ((j * x) % n).double() / n) for j in js for f in (torch.cos, torch.sin)],
                    1).contiguous()
    m, cut = 20, 0.3
    Y = cd.filter(g, X, m, cut, 2.0, 0.0, dtype=dt)
    scale = torch.tensor([_p_m(m, 1 - math.cos(2 * math.pi * j / n), cut) for j in js for _ in (0, 1)],
                         dtype=torch.float64, device=dev)
    err = (Y - X * scale).abs().max().item() / max(1.0, scale.abs().max().item())
    print("cycle modes dt=%d err %.3g" % (dt, err))
    assert err <= tol


@pytest.mark.parametrize("dt,tol", [(0, 1e-12), (1, 1e-4)])
def test_filter_sbm200k_full_size(cd, oracle_mod, dev, dt, tol):
    """The 200k-node, 32-block workload at its filter shape (kb = 32, m = 15)."""
    import torch
    e, n, cfg = synth.make_config_graph("sbm200k")
    g = cd.build_laplacian(e, n)
    o = oracle_mod.build_csr(e, n)
    X = np.random.default_rng(2).standard_normal((n, 32))
    print("case filter sbm200k dt=%d" % dt, flush=True)
    Y = cd.filter(g, torch.from_numpy(X).cuda(), 15, 0.35, 2.0, 0.0, dtype=dt).cpu().numpy()
    want = oracle_mod.cheb_filter(o, X, 15, 0.35)
    err = _rel_err(Y, want)
    print("sbm200k filter dt=%d rel err %.3g" % (dt, err))
    assert err <= tol


# the sparse step keeps 16 neighbour rows in flight per lane (its deep-batch
# form) once the gathered block n x w of the element type exceeds this size
DEEP_BYTES = 256 * 1024 * 1024


@pytest.fixture(scope="module")
def chunglu1m(cd, oracle_mod, dev):
    """The Chung-Lu generator of the 8M-node workload (gamma 2.1, mean degree 16,
    cap sqrt(N), largest component, hubs first) at 1.1M nodes: hub rows of
    degree ~1000 beside rows of degree 1-3, and a 64-wide block larger than
    DEEP_BYTES in FP64 and in FP32, so every step below runs the deep form."""
    e, n = synth.chung_lu(1_100_000, seed=synth.graphs.DEFAULT_SEED + 4)
    return cd.build_laplacian(e, n), oracle_mod.build_csr(e, n)


@pytest.mark.parametrize("dt", [0, 1])
def test_spmm_chung_lu_deep_matches_oracle(cd, oracle_mod, chunglu1m, dt):
    import torch
    g, o = chunglu1m
    kb, es = 64, (8 if dt == 0 else 4)
    assert o.n * kb * es > DEEP_BYTES and int(o.deg.max()) >= 500
    rng = np.random.default_rng(11 + dt)
    npdt = np.float64 if dt == 0 else np.float32
    U = rng.standard_normal((o.n, kb)).astype(npdt)
    Z = rng.standard_normal((o.n, kb)).astype(npdt)
    Ut, Zt = torch.from_numpy(U).cuda(), torch.from_numpy(Z).cuda()
    Yt = torch.empty_like(Ut)
    print("case spmm chung-lu n=%d dt=%d" % (o.n, dt), flush=True)
    AU = oracle_mod.apply_laplacian(o, U.astype(np.float64))
    tol = 1e-14 if dt == 0 else 2e-6
    cd.spmm(g, -1.0, 1.0, 0.0, Ut, None, Yt)
    assert _rel_err(Yt.cpu().numpy().astype(np.float64), AU) <= tol
    a, b, c = 0.7, -1.3, 0.25
    cd.spmm(g, a, b, c, Ut, Zt, Yt)
    U64, Z64 = U.astype(np.float64), Z.astype(np.float64)
    want = a * (U64 - AU) + b * U64 + c * Z64
    assert _rel_err(Yt.cpu().numpy().astype(np.float64), want) <= tol


@pytest.mark.parametrize("dt,tol", [(0, 1e-12), (1, 1e-4)])
def test_filter_chung_lu_deep_matches_oracle(cd, oracle_mod, chunglu1m, dt, tol):
    """All three kinds of filter step (first, interior scaled, last) in the
    deep form, on the hub-heavy graph."""
    import torch
    g, o = chunglu1m
    X = np.random.default_rng(3).standard_normal((o.n, 64))
    print("case filter chung-lu dt=%d" % dt, flush=True)
    Y = cd.filter(g, torch.from_numpy(X).cuda(), 5, 0.3, 2.0, 0.0, dtype=dt).cpu().numpy()
    want = oracle_mod.cheb_filter(o, X, 5, 0.3, 2.0, 0.0)
    err = _rel_err(Y, want)
    print("chung-lu filter dt=%d rel err %.3g" % (dt, err))
    assert err <= tol


def test_filter_rejects_bad_interval(cd, sbm20k):
    import torch
    g, o = sbm20k
    X = torch.zeros(o.n, 4, dtype=torch.float64, device="cuda")
    for args in [(3, 0.0, 2.0, 0.0), (3, 2.5, 2.0, 0.0), (0, 0.5, 2.0, 0.0)]:
        with pytest.raises(cd.ChebdavError) as ei:
            cd.filter(g, X, *args)
        assert ei.value.status == cd.EINVAL
