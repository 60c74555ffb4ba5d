"""Host-side pieces of bench.py (no GPU): the multi-GPU refusal, the
algorithmic flop and byte counts its roofline uses, and the traffic lookup
that reports measured HBM bytes only for the sources they were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2509_02840_amd import bdu  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_applier_flops_are_six_per_rotation_per_row():
    st = bdu.plan_stats(300, 257)
    assert bench.applier_flops(bdu, 300, 257) == 6.0 * (300 * st["left"] + 257 * st["right"])


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_householder_stream_bytes_leading_order(n):
    # per step k the products stream about 4(m + n)k + 3k^2 doubles, so the
    # total is 2(m + n)n^2 + n^3 doubles to leading order (m = n: 5 n^3)
    got = bench.bhu_stream_bytes(n, n) / 8.0
    assert abs(got / (5.0 * n ** 3) - 1.0) < 8.0 / n ** 0.5


def test_traffic_is_reported_only_for_measured_sources():
    t = bench.MEASURED_TRAFFIC
    til = next(iter(t["bytes"]))
    saved = t["sha256"]
    try:
        t["sha256"] = bench.sources_digest()
        assert bench.measured_traffic(t["n"], t["streams"], til) == t["bytes"][til]
    finally:
        t["sha256"] = saved
    assert bench.measured_traffic(t["n"], t["streams"], (12, 3, 1)) is None
    assert bench.measured_traffic(t["n"] + 1, t["streams"], til) is None
    saved = t["sha256"]
    try:
        t["sha256"] = "0" * 64
        assert bench.measured_traffic(t["n"], t["streams"], til) is None
    finally:
        t["sha256"] = saved


@pytest.mark.parametrize("sample", [1, 4])
def test_cpu_baseline_reports_both_modes(sample):
    from paper_2509_02840_amd import workloads as W

    f = W.factorization(96, 64, 11)
    (B, C), = W.gaussian_updates(96, 64, 1, 12)
    out = bench.cpu_baseline(f.Q, f.d, f.e, f.P, B[:, 0], C[:, 0], "a 96x64 stream", single_sample=sample)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] == bench.cpu_threads()
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert out["host"]["logical_cpus"] >= 1
    assert ("extrapolated" in out["single_thread"]["sample"]) == (sample > 1)


def test_cpu_threads_follow_the_thread_cap(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.cpu_threads() == 1
    monkeypatch.setenv("OMP_NUM_THREADS", "")
    assert bench.cpu_threads() == len(os.sched_getaffinity(0))
