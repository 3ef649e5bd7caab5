"""Hand-worked normalized Laplacians of small graphs (Eq. 1), from
tests/golden/laplacian_small.txt: the oracle's CSR pattern, degrees and dense
A against the worked values, its spectrum against the closed forms, and the
GPU graph build against the same CSR, bit for bit."""

import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "laplacian_small.txt")


def _graphs():
    out, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        if key == "graph":
            cur = {"name": rest, "A": []}
        elif key == "end":
            out.append(cur)
        elif key == "n":
            cur["n"] = int(rest)
        elif key == "edges":
            cur["edges"] = [tuple(int(v) for v in t.split("-")) for t in rest.split()]
        elif key in ("row_ptr", "col", "deg"):
            cur[key] = [int(v) for v in rest.split()]
        elif key == "A":
            i, j, v = rest.split()
            cur["A"].append((int(i), int(j), float(v)))
        elif key == "eig":
            cur["eig"] = [float(v) for v in rest.split()]
    return out


GRAPHS = _graphs()


@pytest.mark.parametrize("g", GRAPHS, ids=[g["name"] for g in GRAPHS])
def test_oracle_matches_worked_laplacian(oracle_mod, g):
    csr = oracle_mod.build_csr(np.array(g["edges"]), g["n"])
    assert csr.row_ptr.tolist() == g["row_ptr"]
    assert csr.col.tolist() == g["col"]
    assert csr.deg.tolist() == g["deg"]
    A = oracle_mod.dense_laplacian(csr)
    want = np.eye(g["n"])
    for i, j, v in g["A"]:
        want[i, j] = want[j, i] = v
    assert np.max(np.abs(A - want)) <= 1e-15
    assert np.max(np.abs(np.linalg.eigvalsh(A) - np.array(g["eig"]))) <= 1e-13


@pytest.mark.gpu
@pytest.mark.parametrize("g", GRAPHS, ids=[g["name"] for g in GRAPHS])
def test_gpu_build_matches_worked_csr(cd, dev, g):
    import torch
    gr = cd.build_laplacian(np.array(g["edges"], dtype=np.int64), g["n"])
    rp, col, deg, dinv = cd.graph_export(gr)
    torch.cuda.synchronize()
    row_ptr, col, deg, dinv = rp.cpu().numpy(), col.cpu().numpy(), deg.cpu().numpy(), dinv.cpu().numpy()
    assert row_ptr.tolist() == g["row_ptr"]
    assert col.tolist() == g["col"]
    assert deg.tolist() == g["deg"]
    want = np.array([1.0 / np.sqrt(d) if d > 0 else 0.0 for d in g["deg"]])
    assert np.array_equal(dinv, want)
