"""GPU parity: Laplacian build (Eq. 1) bit-exact against the oracle's CSR,
degrees and dinv; error paths of the build."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _export(cd, g):
    import torch
    rp, col, deg, dinv = cd.graph_export(g)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col.cpu().numpy(), deg.cpu().numpy(), dinv.cpu().numpy()


def _compare(cd, oracle_mod, edges, n, on_device=False):
    import torch
    e = torch.from_numpy(edges).cuda() if on_device else edges
    g = cd.build_laplacian(e, n)
    want = oracle_mod.build_csr(edges, n)
    rp, col, deg, dinv = _export(cd, g)
    assert g.n == n and g.nnz == want.nnz
    assert np.array_equal(rp, want.row_ptr)
    assert np.array_equal(col, want.col)
    assert np.array_equal(deg, want.deg)
    assert np.array_equal(dinv.view(np.uint64), want.dinv.view(np.uint64))   # bit-exact
    assert g.n_isolated == int((want.deg == 0).sum())
    assert g.max_deg == int(want.deg.max(initial=0))
    return g


def test_sbm5k(cd, oracle_mod, dev):
    e, n, _ = synth.make_config_graph("sbm5k")
    print("case sbm5k", flush=True)
    _compare(cd, oracle_mod, e, n)


def test_duplicates_loops_isolated_both_orientations(cd, oracle_mod, dev):
    rng = np.random.default_rng(3)
    n = 3001
    raw = rng.integers(0, n - 5, size=(20000, 2))       # last 5 nodes isolated
    raw = np.concatenate([raw, raw[:5000, ::-1], raw[5000:7000], np.stack([np.arange(50)] * 2, 1)])
    print("case dupes", flush=True)
    _compare(cd, oracle_mod, raw.astype(np.int64), n)
    _compare(cd, oracle_mod, raw.astype(np.int64), n, on_device=True)


def test_all_row_length_bins(cd, oracle_mod, dev):
    # rows of length <= 64, (64, 4096] and > 4096 (a hub of 10000 + duplicates)
    parts = [(synth.star_graph(10001), 10001), (synth.star_graph(3000), 3000),
             (synth.star_graph(65), 65), (synth.star_graph(64), 64), (synth.cycle_graph(1000), 1000),
             (synth.complete_graph(80), 80)]
    e, n = synth.disjoint_union(parts)
    e = np.concatenate([e, e[:4000, ::-1]])
    print("case bins", flush=True)
    _compare(cd, oracle_mod, e, n)


def test_chung_lu_skewed(cd, oracle_mod, dev):
    e, n = synth.chung_lu(200_000, seed=11)
    print("case chung-lu", flush=True)
    _compare(cd, oracle_mod, e, n)


def test_sbm200k(cd, oracle_mod, dev):
    e, n, _ = synth.make_config_graph("sbm200k")
    print("case sbm200k", flush=True)
    _compare(cd, oracle_mod, e, n)


def test_empty_and_tiny(cd, oracle_mod, dev):
    _compare(cd, oracle_mod, np.zeros((0, 2), dtype=np.int64), 5)
    _compare(cd, oracle_mod, np.array([[0, 0]], dtype=np.int64), 1)
    _compare(cd, oracle_mod, np.array([[0, 1]], dtype=np.int64), 2)


def test_invalid_inputs(cd, dev):
    with pytest.raises(cd.ChebdavError) as ei:
        cd.build_laplacian(np.array([[0, 5]], dtype=np.int64), 5)
    assert ei.value.status == cd.EINVAL
    with pytest.raises(cd.ChebdavError) as ei:
        cd.build_laplacian(np.array([[-1, 2]], dtype=np.int64), 5)
    assert ei.value.status == cd.EINVAL
    with pytest.raises(cd.ChebdavError) as ei:
        cd.build_laplacian(np.zeros((0, 2), dtype=np.int64), 0)
    assert ei.value.status == cd.EINVAL


def test_dinv_exhaustive(cd, dev):
    """Every degree 1..10^7: the device arithmetic equals 1/sqrt in IEEE
    round-to-nearest (NumPy's, itself pinned by exact rational arithmetic)."""
    import torch
    d = torch.arange(0, 10_000_001, dtype=torch.int32, device=dev)
    got = cd.dinv(d).cpu().numpy()
    dd = np.arange(0, 10_000_001, dtype=np.float64)
    want = np.zeros_like(dd)
    want[1:] = 1.0 / np.sqrt(dd[1:])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("case", ["chung_lu", "sbm", "tiny"])
def test_row_split_covers_rows_and_balances(cd, oracle_mod, dev, case):
    """chebdav_graph_row_split: nine non-decreasing boundaries from 0 to n (the
    eight per-XCD row ranges of the sparse step); on a large graph every range
    carries about one eighth of nnz + 4 rows (largest range within 10 % of the
    mean, or within one row's weight of it)."""
    if case == "chung_lu":
        e, n = synth.chung_lu(200_000, seed=5)
    elif case == "sbm":
        e, _ = synth.sbm(100_000, 16, d_in=20, d_out=4, uneven=True, seed=6)
        n = 100_000
    else:
        e, n = synth.path_graph(5), 5
    g = cd.build_laplacian(e, n)
    b = np.array(cd.graph_row_split(g))
    assert b[0] == 0 and b[-1] == n and (np.diff(b) >= 0).all()
    if case != "tiny":
        o = oracle_mod.build_csr(e, n)
        w = np.diff(o.row_ptr) + 4
        cw = np.concatenate([[0], np.cumsum(w)])
        per = cw[b[1:]] - cw[b[:-1]]
        assert per.max() <= max(1.1 * cw[-1] / 8, cw[-1] / 8 + w.max())
