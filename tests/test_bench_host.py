"""Host-side contract of bench.py, on the CPU: the one-GPU refusal, the
latency percentile, and when the committed HBM-traffic figure is reported."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    # exits before anything touches a GPU
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_percentile_is_nearest_rank(bench):
    rng = np.random.default_rng(3)
    for n in (1, 2, 7, 100, 1001):
        x = rng.exponential(size=n).tolist()
        for q in (1, 50, 90, 99, 100):
            assert bench.percentile(x, q) == pytest.approx(np.percentile(x, q, method="inverted_cdf"))
    assert bench.percentile([], 50) is None


def test_traffic_only_for_the_profiled_kernel_and_workload(bench):
    path = os.path.join(ROOT, "profiles", "k_join_c3_traffic.json")
    with open(path) as fh:
        rec = json.load(fh)
    t = rec["t"]
    # never at a reduced size, and never at another threshold
    assert bench.measured_traffic("c3", t, 300000) is None
    assert bench.measured_traffic("c3", t + 0.05, None) is None
    # at full size: the stored figure while the summary was taken on the
    # kernel source as it is, else nothing
    got = bench.measured_traffic("c3", t, None)
    if rec["source_hash"] == bench.kernel_source_hash():
        assert got == rec["traffic_bytes"]
        assert got > 0
    else:
        assert got is None
    # a workload with no counter summary
    assert bench.measured_traffic("c1", 0.5, None) is None
