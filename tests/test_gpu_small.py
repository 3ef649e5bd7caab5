"""GPU units: the small symmetric eigensolver (Alg. 2 step 9) against LAPACK
(numpy.linalg.eigh), and the Philox generator bit-exact against the oracle's."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _check_eig(cd, H, tol_val=1e-12):
    import torch
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    w, Y = cd.small_eig(Ht)
    w, Y = w.cpu().numpy(), Y.cpu().numpy()
    n = H.shape[0]
    ref = np.linalg.eigvalsh(H)
    nrm = max(np.abs(ref).max(), 1e-300)
    assert (np.diff(w) >= 0).all()
    assert np.abs(w - ref).max() <= tol_val * nrm, np.abs(w - ref).max() / nrm
    assert np.linalg.norm(H @ Y - Y * w, 2) <= 1e-12 * nrm * max(1, np.sqrt(n) / 4)
    assert np.linalg.norm(Y.T @ Y - np.eye(n), 2) <= 1e-13 * max(1, np.sqrt(n) / 4)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16, 17, 30, 33, 64, 65, 97, 128, 129, 159, 160, 161, 320, 448])
def test_random_symmetric(cd, dev, n):
    A = np.random.default_rng(n).standard_normal((n, n))
    print("case eig random n=%d" % n, flush=True)
    _check_eig(cd, (A + A.T) / 2)


@pytest.mark.parametrize("n,kb", [(38, 4), (160, 32), (320, 64)])
def test_arrowhead(cd, dev, n, kb):
    """The Rayleigh-quotient shape after a restart: diagonal plus a kb-wide border."""
    rng = np.random.default_rng(kb)
    H = np.diag(np.sort(rng.uniform(0.0, 2.0, n)))
    B = 1e-3 * rng.standard_normal((n, kb))
    H[:, n - kb:] += B
    H[n - kb:, :] += B.T
    H = (H + H.T) / 2
    print("case eig arrowhead n=%d" % n, flush=True)
    _check_eig(cd, H)


@pytest.mark.parametrize("n", [10, 100, 150, 200])
def test_degenerate(cd, dev, n):
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat(np.array([0.0, 0.25, 0.25 + 1e-14, 1.0, 2.0]), n // 5)
    print("case eig degenerate n=%d" % n, flush=True)
    _check_eig(cd, (Q * lam) @ Q.T)


def test_diagonal_and_zero(cd, dev):
    _check_eig(cd, np.diag(np.array([3.0, -1.0, 2.0, 2.0, 0.5])))
    _check_eig(cd, np.diag(np.linspace(0.1, 1.9, 100)))
    import torch
    w, Y = cd.small_eig(torch.zeros(6, 6, dtype=torch.float64, device="cuda"))
    assert np.abs(w.cpu().numpy()).max() <= 1e-300
    Yn = Y.cpu().numpy()
    assert np.linalg.norm(Yn.T @ Yn - np.eye(6)) < 1e-13


def test_philox_bit_exact(cd, oracle_mod, dev):
    seed = (123 << 32) | 456
    X = cd.philox_fill(5000, 7, seed, first_col=40).cpu().numpy()
    want = oracle_mod.random_block(seed, 5000, np.arange(40, 47))
    assert np.array_equal(X.view(np.uint64), np.ascontiguousarray(want).view(np.uint64))
