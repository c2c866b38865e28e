"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and
the rule that a committed traffic figure is reported only for the kernel
sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figure_follows_the_kernel_sources():
    wl = "c2_chain_ar1_n1000_p10000_f32"
    for k in ("gemv_a", "gemv_b"):
        with open(os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (k, wl))) as fh:
            t = json.load(fh)
        got = bench.measured_traffic(k, wl)
        if t["kernel_source_hash"] == bench.kernel_source_hash():
            assert got == t["bytes_per_launch"]
            # counters scaled by the plain-copy factors: reads and writes add up
            assert abs(t["read_bytes"] + t["write_bytes"] - got) <= 1e-6 * got
        else:
            assert got is None
    assert bench.measured_traffic("gemv_a", "no_such_workload") is None
