"""GPU: blocks whose shape, dtype or device does not match the graph or the
other arguments are refused by the binding (ValueError) before the library
sees their pointers."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_mismatched_blocks_refused(cd, dev):
    import torch
    n = 2000
    e, _ = synth.sbm(n, 4, d_in=10, d_out=2, seed=3)
    g = cd.build_laplacian(e, n)
    short = torch.zeros(n - 1, 4, dtype=torch.float64, device="cuda")
    ok = torch.zeros(n, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError, match="rows"):
        cd.filter(g, short, 5, 0.5)
    with pytest.raises(ValueError, match="rows"):
        cd.solve(g, cd.make_params(k_want=4, kb=4, m=11), V_init=short)
    with pytest.raises(ValueError, match="float64"):
        cd.filter(g, ok.float(), 5, 0.5)
    with pytest.raises(ValueError, match="columns"):
        cd.spmm(g, -1.0, 1.0, 0.0, ok, None, torch.zeros(n, 3, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="rows"):
        cd.orthonormalize(short, ok)
    with pytest.raises(ValueError, match="rows"):
        cd.rayleigh_ritz(g, torch.zeros(n + 1, 4, dtype=torch.float32, device="cuda"))
    # the well-formed call still runs
    Y = cd.filter(g, torch.randn(n, 4, dtype=torch.float64, device="cuda"), 5, 0.5)
    assert np.isfinite(Y.cpu().numpy()).all()
