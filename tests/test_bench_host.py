"""Host-side pieces of the benchmark script: the algorithmic flop counts
that the roofline fraction divides by (hand-computed values), the traffic
figure's source-hash gate, and the one-GPU argument check."""

import json
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_coefficient_flops_hand_case():
    # 3->4->5->1: one hidden product (layer 2, 5 x 4) over D = 3 symbols + centre
    assert bench.alg_flops_coefficient([3, 4, 5, 1]) == 2 * 5 * 4 * 4
    # 3->4->5->6->1: layer 3 (6 x 5) over D = 3 + 4 symbols + centre
    assert bench.alg_flops_coefficient([3, 4, 5, 6, 1]) == 2 * 5 * 4 * 4 + 2 * 6 * 5 * 8


def test_covariance_hybrid_flops_on_the_256x5_net():
    # layers 2, 3 in coefficient form (2*256^2*3, 2*256^2*259), layer 4 builds
    # Sigma (256^2*515) and switches, layers 4, 5 pay 3*256^3 each
    n = 256
    want = 2 * n * n * 3 + 2 * n * n * 259 + n * n * 515 + 2 * 3 * n ** 3
    got = bench.alg_flops_cov_hybrid([3, n, n, n, n, n, 1])
    assert got == want
    assert got == pytest.approx(168.75e6, rel=1e-3)


def test_traffic_figure_needs_the_profiled_source():
    t = json.loads((ROOT / "profiles" / "hidden_cov_bf16_traffic.json").read_text())
    assert set(t) >= {"kernel_source_sha256_16", "hbm_bytes_per_cell"}
    if t["kernel_source_sha256_16"] == bench.kernel_source_hash("hidden_cov_bf16"):
        assert bench.traffic_from_profiles("hidden_cov_bf16", 1000.0) == pytest.approx(1000.0 * t["hbm_bytes_per_cell"])
    else:
        assert bench.traffic_from_profiles("hidden_cov_bf16", 1000.0) is None


def test_traffic_figure_is_dropped_for_another_source(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kind, src=None: "0" * 16)
    assert bench.traffic_from_profiles("hidden_cov_bf16", 1000.0) is None


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus must be 1" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
