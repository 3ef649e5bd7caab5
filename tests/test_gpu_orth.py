"""GPU: block orthonormalization (Alg. 2 step 6) by its invariants, and the
replacement of exactly dependent columns (same count as the oracle's DGKS)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _basis(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return np.ascontiguousarray(q)


def _run(cd, V, X, seed=0, first=0):
    import torch
    Vt = torch.from_numpy(V).cuda() if V is not None and V.shape[1] else None
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    rep = cd.orthonormalize(Vt, Xt, seed=seed, first_random_col=first)
    return Xt.cpu().numpy(), rep


@pytest.mark.parametrize("n,ksub,kb", [(2000, 40, 8), (50_000, 224, 32), (100_000, 384, 64), (777, 0, 5)])
def test_invariants_and_span(cd, dev, n, ksub, kb):
    V = _basis(n, ksub, 0) if ksub else np.zeros((n, 0))
    X = np.random.default_rng(1).standard_normal((n, kb))
    print("case orth n=%d ksub=%d kb=%d" % (n, ksub, kb), flush=True)
    Q, rep = _run(cd, V, X)
    assert rep == 0
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    if ksub:
        assert np.linalg.norm(V.T @ Q, 2) <= 10 * ksub * EPS
    Xp = X - V @ (V.T @ X) if ksub else X
    assert np.linalg.norm(Xp - Q @ (Q.T @ Xp)) <= 1e-12 * np.linalg.norm(Xp)


def test_ill_conditioned_mostly_in_span(cd, dev):
    n, kb = 3000, 6
    V = _basis(n, 20, 4)
    base = np.random.default_rng(5).standard_normal((n, 1))
    X = base + 1e-5 * np.random.default_rng(6).standard_normal((n, kb))
    X = X + V @ np.random.default_rng(7).standard_normal((20, kb)) * 1e3
    Q, rep = _run(cd, V, X)
    assert rep == 0
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 100 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 100 * 20 * EPS
    Xp = X - V @ (V.T @ X)
    assert np.linalg.norm(Xp - Q @ (Q.T @ Xp)) <= 1e-9 * np.linalg.norm(Xp)


def _kahan(kb, s):
    """Kahan's upper-triangular matrix diag(1, s, .., s^(kb-1)) (I - c U), c^2 + s^2 = 1,
    U the strictly upper ones: unit-norm columns, scaled pivots s^j, and a
    condition number growing like ((1 + c)/s)^kb."""
    c = np.sqrt(1.0 - s * s)
    return np.diag(s ** np.arange(kb)) @ (np.eye(kb) - c * np.triu(np.ones((kb, kb)), 1))


@pytest.mark.parametrize("method", ["cholqr", "tsqr"])
def test_graded_block_pivots_above_threshold(cd, dev, method):
    """A graded block whose scaled Cholesky pivots all stay >= 0.01 but whose
    condition number is 1.2e5 (Kahan's matrix, kb = 16): the first Cholesky QR
    alone would leave X^T X about kappa^2 eps away from I and V^T X about kappa
    eps, so the orthonormalizer must take its full second pass."""
    n, ksub, kb = 20_000, 48, 16
    V = _basis(n, ksub, 21)
    K = _kahan(kb, 0.78)
    assert (0.78 ** np.arange(kb)).min() >= 0.01 and np.linalg.cond(K) >= 1e5
    Q0 = _basis(n, ksub + kb, 22)[:, ksub:]
    Q0 = Q0 - V @ (V.T @ Q0)
    Q0, _ = np.linalg.qr(Q0)
    X = Q0 @ K + V @ np.random.default_rng(23).standard_normal((ksub, kb))
    print("case graded block %s" % method, flush=True)
    Q, rep = _run_m(cd, V, X, method)
    assert rep == 0
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 10 * ksub * EPS
    Xp = X - V @ (V.T @ X)
    assert np.linalg.norm(Xp - Q @ (Q.T @ Xp)) <= 1e-10 * np.linalg.norm(Xp)


def _run_m(cd, V, X, method):
    import torch
    Vt = torch.from_numpy(V).cuda()
    Xt = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    rep = cd.orthonormalize(Vt, Xt, method=method)
    return Xt.cpu().numpy(), rep


def test_exactly_dependent_columns(cd, oracle_mod, dev):
    n, kb = 1500, 6
    V = _basis(n, 10, 8)
    X = np.random.default_rng(9).standard_normal((n, kb))
    X[:, 2] = X[:, 0]
    X[:, 4] = V @ np.arange(1.0, 11.0)
    X[:, 5] = 0.0
    Q, rep = _run(cd, V, X, seed=2, first=100)
    _, rep_oracle, _ = oracle_mod.dgks(np.asfortranarray(V), X, seed=2, next_col=100)
    assert rep == rep_oracle == 3
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 100 * EPS
    # the independent columns keep their span
    keep = X[:, [0, 1, 3]] - V @ (V.T @ X[:, [0, 1, 3]])
    assert np.linalg.norm(keep - Q @ (Q.T @ keep)) <= 1e-12 * np.linalg.norm(keep)


@pytest.mark.parametrize("n,ksub,kb,ldv,ldx,offv,offx",
                         [(3001, 37, 33, 41, 35, 3, 1), (4099, 150, 64, 151, 66, 0, 2), (2500, 16, 17, 16, 18, 0, 1)])
def test_strided_unaligned_views(cd, dev, n, ksub, kb, ldv, ldx, offv, offx):
    """V and X as column windows of wider arrays (odd leading dimensions, bases
    not 16-byte aligned): same invariants, and the columns beside the window
    are left untouched."""
    import torch
    print("case orth views n=%d ksub=%d kb=%d ldv=%d ldx=%d" % (n, ksub, kb, ldv, ldx), flush=True)
    V = _basis(n, ksub, 11)
    X = np.random.default_rng(12).standard_normal((n, kb))
    Vbig = np.random.default_rng(13).standard_normal((n, ldv + offv))
    Vbig[:, offv:offv + ksub] = V
    Xbig = np.random.default_rng(14).standard_normal((n, ldx + offx))
    Xbig[:, offx:offx + kb] = X
    Vb = torch.from_numpy(Vbig).cuda()
    Xb = torch.from_numpy(Xbig).cuda()
    rep = cd.orthonormalize(Vb[:, offv:offv + ksub], Xb[:, offx:offx + kb], seed=0)
    out = Xb.cpu().numpy()
    Q = out[:, offx:offx + kb]
    assert rep == 0
    assert np.array_equal(np.delete(out, np.s_[offx:offx + kb], axis=1), np.delete(Xbig, np.s_[offx:offx + kb], axis=1))
    assert np.array_equal(Vb.cpu().numpy(), Vbig)
    assert np.linalg.norm(Q.T @ Q - np.eye(kb), 2) <= 10 * kb * EPS
    assert np.linalg.norm(V.T @ Q, 2) <= 10 * ksub * EPS
    Xp = X - V @ (V.T @ X)
    assert np.linalg.norm(Xp - Q @ (Q.T @ Xp)) <= 1e-12 * np.linalg.norm(Xp)


def test_argument_errors_launch_nothing(cd, dev):
    """Rejected calls return their status before any kernel runs: block wider
    than 64 columns, no room for an orthonormal block, unknown method, NULL or
    short workspace (orthonormalizer and small eigensolver)."""
    import ctypes
    import torch
    L = cd._lib
    n, ksub = 1000, 8
    V = torch.zeros((n, ksub), dtype=torch.float64, device="cuda")
    X = torch.zeros((n, 70), dtype=torch.float64, device="cuda")
    rep = ctypes.c_int(-1)
    null = ctypes.c_void_p(0)

    def orth(kb, nn, method, ws, ws_bytes, ks=ksub):
        return L.chebdav_orthonormalize(ctypes.c_void_p(V.data_ptr()), ksub, ks, ctypes.c_void_p(X.data_ptr()),
                                        70, kb, nn, 0, 0, method, ctypes.byref(rep), ws, ws_bytes, null)

    need = ctypes.c_size_t()
    assert L.chebdav_orthonormalize_workspace_size(n, ksub, 16, cd.ORTH_CHOLQR, ctypes.byref(need)) == cd.OK
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    wsp = ctypes.c_void_p(ws.data_ptr())
    assert orth(65, n, cd.ORTH_CHOLQR, wsp, need.value) == cd.EUNSUPPORTED
    assert orth(16, 20, cd.ORTH_CHOLQR, wsp, need.value) == cd.EINVAL  # n < ksub + kb
    assert orth(16, n, 7, wsp, need.value) == cd.EINVAL
    assert orth(16, n, cd.ORTH_CHOLQR, null, need.value) == cd.ENOMEM
    assert orth(16, n, cd.ORTH_CHOLQR, wsp, need.value - 1) == cd.ENOMEM
    assert rep.value == -1  # untouched on error
    H = torch.eye(40, dtype=torch.float64, device="cuda")
    w = torch.empty(40, dtype=torch.float64, device="cuda")
    Y = torch.empty((40, 40), dtype=torch.float64, device="cuda")
    assert L.chebdav_small_eig(ctypes.c_void_p(H.data_ptr()), 40, 40, ctypes.c_void_p(w.data_ptr()),
                               ctypes.c_void_p(Y.data_ptr()), 40, null, 1 << 30, null) == cd.ENOMEM
    torch.cuda.synchronize()
