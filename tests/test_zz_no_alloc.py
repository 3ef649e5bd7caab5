"""GPU: chebdav_filter_noalloc (the filter on the library's static scratch)
against chebdav_filter with a caller workspace, through the C ABI.  Both run
the same kernels on the same inputs, so the outputs must be identical bit for
bit; two calls in a row, the second on a smaller graph and block, show that the
buffer's leftover contents from the first call do not leak into the second.
Also checked: a shape beyond the static buffer is rejected before any launch."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [0, 1])
def test_noalloc_filter_matches_workspace_filter(cd, oracle_mod, dev, dt):
    import torch
    cases = [(20_000, 16, 32, 15, 0.35, 7), (5_000, 4, 8, 11, 0.2, 8)]   # second: smaller graph and block
    for n, B, kb, m, cut, seed in cases:
        e, _ = synth.sbm(n, B, d_in=18, d_out=3, uneven=True, seed=seed)
        g = cd.build_laplacian(e, n)
        X = torch.from_numpy(np.random.default_rng(seed).standard_normal((n, kb))).cuda()
        print("case noalloc filter n=%d kb=%d m=%d dt=%d" % (n, kb, m, dt), flush=True)
        Y0 = cd.filter(g, X, m, cut, 2.0, 0.0, dtype=dt)
        Y1 = torch.full_like(X, float("nan"))
        cd.filter_noalloc(g, X, m, cut, 2.0, 0.0, dtype=dt, Y=Y1)
        torch.cuda.synchronize()
        assert torch.equal(Y0, Y1)
        want = oracle_mod.cheb_filter(oracle_mod.build_csr(e, n), X.cpu().numpy(), m, cut, 2.0, 0.0)
        err = float(np.abs(Y1.cpu().numpy() - want).max() / np.abs(want).max())
        assert err <= (1e-12 if dt == 0 else 1e-4)


def test_noalloc_filter_rejects_oversized_block(cd, dev):
    import torch
    n = 300_000
    g = cd.build_laplacian(synth.cycle_graph(n), n)
    X = torch.zeros(n, 32, dtype=torch.float64, device="cuda")   # 3 x 76.8 MB > 64 MiB
    with pytest.raises(cd.ChebdavError) as ei:
        cd.filter_noalloc(g, X, 5, 0.5)
    assert ei.value.status == cd.EUNSUPPORTED
