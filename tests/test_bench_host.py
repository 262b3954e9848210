"""Host-side pieces of the benchmark: the algorithmic flop count behind the
split form's roofline, the traffic figure read from the committed counter
summary (and dropped when the kernel sources have changed), and the refusal
of runs on several GPUs."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_split_flop_count_per_element():
    # 3 directions x 16 lines x 6 unordered pairs x (70 + 20) operations
    assert bench.split_flops_per_element(3, 3) == 3 * 16 * 6 * 90 == 25920
    # 2-D, N = 1: 2 directions x 2 lines x 1 pair x (65 + 16)
    assert bench.split_flops_per_element(2, 1) == 2 * 2 * 1 * 81
    assert abs(bench.split_flops_per_element(3, 3) * 32 ** 3 / 1e9 - 0.849) < 1e-3


def test_traffic_follows_the_committed_counters():
    path = os.path.join(ROOT, "profiles", "k_stage_n3_euler3d_f64_counters.json")
    with open(path) as fh:
        c = json.load(fh)
    alg = bench.WORDS_PER_DOF_STAGE * 8 * 32 ** 3 * 64 * 5
    t = bench.measured_traffic(alg)
    if c["source_sha256"] != bench.kernel_source_hash():
        assert t is None
        pytest.skip("kernel sources changed since the counters were taken")
    want = (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0
    assert t["bytes_per_launch"] == pytest.approx(want)
    assert t["over_algorithmic"] == pytest.approx(want / alg)
    # the calibration: a plain copy of 512 MiB reads and writes 512 MiB
    assert c["fetch_scale"] * c["copy_fetch_kib"] == pytest.approx(c["copy_kib"])
    assert c["write_scale"] * c["copy_write_kib"] == pytest.approx(c["copy_kib"])


def test_traffic_dropped_when_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(1.0) is None


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
