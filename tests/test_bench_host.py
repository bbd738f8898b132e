"""Host logic of bench.py (no GPU): the one-GPU rule, the algorithmic byte
counts of the roofline, and the rule that HBM traffic is reported only from a
counter summary taken on the current kernel source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_bytes_per_unit():
    st = {"nnz_L": 1000, "nnz_P": 300, "adj_factor_bytes": 50000}
    m, E, K, T = 100, 261, 20, 3
    C = [0, 10, 20]
    fwd, bwd_d = bench.algorithmic_bytes(st, m, E, C, K, T, adj_iters=4, direct=True)
    per_iter = 2 * 1000 * 12 + 4 * 300 * 8 + 261 * 16 + 100 * 12
    assert fwd == T * (K * per_iter + 300 * 12 + 100 * 24) + K * 30 * 48
    assert bwd_d == 4 * (50000 + 4 * 300 * 8 + 300 * 12 + 261 * 16 + 6 * 300 * 8 + 10 * 72)
    _, bwd_i = bench.algorithmic_bytes(st, m, E, C, K, T, adj_iters=4, direct=False)
    assert bwd_i == 4 * (2 * 1000 * 12 + 300 * 12 + 261 * 16 + 6 * 300 * 8 + 10 * 72)


def test_traffic_only_for_the_current_source(tmp_path, monkeypatch):
    src = (
        "kernel_source_sha256_16: {h}  (kernels.hip + capi.cpp)\n"
        "k_forward_hbm_bytes_per_launch: 1.5e+07\n")
    p = tmp_path / "pmc.txt"
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(p))
    p.write_text(src.format(h=bench.source_hash()))
    assert bench.traffic_from_profile("k_forward") == 1.5e7
    assert bench.traffic_from_profile("k_backward") is None
    p.write_text(src.format(h="0" * 16))
    assert bench.traffic_from_profile("k_forward") is None
