"""bench.py's command line on the host: more than one GPU is refused with a
message (the segmentation of one field runs on one device), and the
algorithmic-byte accounting and traffic lookup behave as documented."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes():
    assert bench.algo_bytes("jump", 1) == 16.0  # U, D read; desc, asc written (the record index is overhead)
    assert bench.algo_bytes("steepest", 1) == 12.0
    assert bench.algo_bytes("order_last", 1) == 16.0 and bench.algo_bytes("order_last", 2) == 12.0
    assert bench.algo_bytes("order_invert", 4) == 5.0
    assert bench.algo_bytes("radix_scatter", 1) is None


def test_profile_lookup_guards():
    for name in ("hbm_traffic", "kernel_stats"):
        assert bench.profile_entry(name, "no_such_workload", "jump", {})[0] is None
        # a knob setting other than the profiled one yields no figure
        t, why = bench.profile_entry(name, "c3", "jump", {"scan_depth": 8, "scan_rounds": 3})
        assert t is None and why


def test_step_stats_drop_best_and_worst():
    st = bench.step_stats([5.0, 1.0, 2.0, 3.0, 100.0])
    assert st["trimmed_mean_ms"] == 10.0 / 3 and st["median_ms"] == 3.0
    assert st["min_ms"] == 1.0 and st["max_ms"] == 100.0
