"""Host-side parts of bench.py: the one-GPU guard and the rule that counter-derived traffic
is reported only for the kernel source and launch configuration it was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_the_measured_configuration(monkeypatch):
    import hashlib
    with open(bench.KERNELS_SRC, "rb") as f:
        monkeypatch.setitem(bench.TRAFFIC, "sha256", hashlib.sha256(f.read()).hexdigest())
    t = dict(bench.TRAFFIC)
    ok = bench.measured_traffic(t["workload"], t["precision"], t["h_tile"], t["group_max"], "n_f64")
    assert ok == t["bytes_per_launch"]["n_f64"]
    assert bench.measured_traffic("block100", t["precision"], t["h_tile"], t["group_max"], "n_f64") is None
    assert bench.measured_traffic(t["workload"], "fp32", t["h_tile"], t["group_max"], "n_f64") is None
    assert bench.measured_traffic(t["workload"], t["precision"], 128, t["group_max"], "n_f64") is None
    assert bench.measured_traffic(t["workload"], t["precision"], t["h_tile"], 192, "n_f64") is None
    # a different kernel source invalidates the figure
    monkeypatch.setitem(bench.TRAFFIC, "sha256", "0" * 64)
    assert bench.measured_traffic(t["workload"], t["precision"], t["h_tile"], t["group_max"], "n_f64") is None
