"""Host-side logic of bench.py (no GPU): the algorithmic bytes of the sparse
step, and the rule that the measured HBM traffic is reported only while the
stored counter summary was taken on the current kernel source."""

import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bytes_per_step_formula():
    # sbm200k: CSR pattern 4 nnz + row_ptr 8 (n+1) + dinv 8 n + three n x kb FP64 blocks
    n, nnz, kb = 200_000, 4_802_318, 32
    assert bench.bytes_per_step(n, nnz, kb, 8) == 4 * nnz + 8 * (n + 1) + 8 * n + 3 * n * kb * 8 == 176_009_280
    # FP32 blocks and dinv32
    assert bench.bytes_per_step(n, nnz, kb, 4) == 4 * nnz + 8 * (n + 1) + 4 * n + 3 * n * kb * 4


def test_committed_traffic_matches_kernel_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_cheb_step_sbm200k_traffic.json")))
    src = open(os.path.join(ROOT, "paper_2212_04443_amd", "csrc", "spmm.hip"), "rb").read()
    assert rec["source_sha256"] == hashlib.sha256(src).hexdigest()
    t = bench.measured_traffic("sbm200k", bench.step_kernel_name(200_000, 32, 8))
    assert t is not None and 1e8 < t < 1e9


def test_traffic_dropped_when_source_differs(tmp_path, monkeypatch):
    # a copy of the tree whose kernel source differs from the one the counters were taken on
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2212_04443_amd" / "csrc").mkdir(parents=True)
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_cheb_step_sbm200k_traffic.json")))
    (tmp_path / "profiles" / "k_cheb_step_sbm200k_traffic.json").write_text(json.dumps(rec))
    (tmp_path / "paper_2212_04443_amd" / "csrc" / "spmm.hip").write_text("// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k = bench.step_kernel_name(200_000, 32, 8)
    assert bench.measured_traffic("sbm200k", k) is None
    assert bench.measured_traffic("no_such_workload", k) is None


def test_kernel_name_follows_the_launch_rule():
    # 16 bytes per lane, G = lanes rounded up to a power of two, deep batches
    # once the gathered block exceeds 256 MiB
    assert bench.step_kernel_name(200_000, 32, 8) == "k_cheb_step<double, double, 2, 16, false, false>"
    assert bench.step_kernel_name(7_857_986, 64, 8) == "k_cheb_step<double, double, 2, 32, false, true>"
    assert bench.step_kernel_name(7_857_986, 64, 4) == "k_cheb_step<float, float, 4, 16, false, true>"
    assert bench.step_kernel_name(1_000_000, 64, 4) == "k_cheb_step<float, float, 4, 16, false, false>"
    assert bench.step_kernel_name(2_000_000, 40, 8) == "k_cheb_step<double, double, 2, 32, false, true>"
    assert bench.step_kernel_name(100, 3, 8) == "k_cheb_step<double, double, 1, 4, false, false>"
    assert bench.step_kernel_name(100, 6, 4) == "k_cheb_step<float, float, 1, 8, false, false>"
