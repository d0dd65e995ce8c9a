"""bench.py's command line on the CPU: more than one GPU is refused with a
message, and the kernel-source hash that guards the profiled traffic figure
is stable."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_figure_is_tied_to_the_kernel_sources_and_the_workload():
    """A committed counter figure is used only by a run of the same kernel
    sources and the same workload key (configuration and step window)."""
    import argparse
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_source_sha()
    assert len(sha) == 16 and sha == bench.kernel_source_sha()
    args = argparse.Namespace(lanes="none", dtype="f64", eps=1e-4, theta=0.8, theta_zz=-1.5707963267948966,
                              trunc="magnitude", warmup=18, steps=2)
    key = bench.workload_key(args)
    assert key == ("lanes=none dtype=f64 eps=0.0001 theta=0.8 theta_zz=-1.570796 trunc=magnitude "
                   "steps=19-20")
    traffic, alg, src = bench.measured_traffic(key)
    if traffic is not None:  # a summary taken on these sources and this workload
        assert src.startswith("k_rx_merge__") and 1e8 < traffic < 1e11 and 0.9 < traffic / alg < 3.0
    other = argparse.Namespace(**{**vars(args), "warmup": 5})
    assert bench.measured_traffic(bench.workload_key(other)) == (None, None, None)
