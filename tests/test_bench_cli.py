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


def test_traffic_figure_is_tied_to_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_source_sha()
    assert len(sha) == 16 and sha == bench.kernel_source_sha()
    traffic, src = bench.measured_traffic()
    if traffic is not None:  # a summary taken on these sources: a plausible per-launch byte count
        assert src.startswith("k_rx_merge__") and 1e8 < traffic < 1e11
