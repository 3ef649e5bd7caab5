"""GPU: chebdav_filter_noalloc under HIP graph capture, the use it exists for.
The filter (every launch on the caller's stream, no allocation, no memset, no
synchronization) is captured once into a graph; each replay must equal the
eager workspace filter of whatever the input buffer holds at that moment, with
eager work and synchronizations between the replays."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [0, 1])
def test_noalloc_filter_replays_in_a_graph(cd, dev, dt):
    import torch
    n, kb, m, cut = 20_000, 16, 11, 0.3
    e, _ = synth.sbm(n, 8, d_in=14, d_out=3, uneven=True, seed=12)
    g = cd.build_laplacian(e, n)
    X = torch.empty(n, kb, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    X.copy_(torch.from_numpy(np.random.default_rng(0).standard_normal((n, kb))))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        cd.filter_noalloc(g, X, m, cut, 2.0, 0.0, dtype=dt, Y=Y, stream=s)  # first call on this GPU: buffer lookup
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    print("case graph capture of the no-alloc filter dt=%d" % dt, flush=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        cd.filter_noalloc(g, X, m, cut, 2.0, 0.0, dtype=dt, Y=Y, stream=s)
    torch.cuda.synchronize()
    for r in range(4):
        X.copy_(torch.from_numpy(np.random.default_rng(100 + r).standard_normal((n, kb))))
        Y.fill_(float("nan"))
        want = cd.filter(g, X, m, cut, 2.0, 0.0, dtype=dt)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, want), "replay %d differs from the eager filter" % r
