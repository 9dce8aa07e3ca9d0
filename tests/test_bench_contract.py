"""bench.py's contract on a machine without a GPU: a multi-GPU request is
refused with a message, and the committed HBM-counter summaries belong to
the tau-stream kernel as it is now (a kernel change without new counters
would silently drop the traffic field from the bench line)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_counters_match_the_stream_kernel():
    for mixed in (False, True):
        t = bench.stream_traffic(mixed)
        assert t is not None, "profiles/traffic_tau_stream_*.json was taken on another kernel"
        # more than the algorithmic tau bytes of one C2 launch, less than twice
        algo = (4 if mixed else 8) * 93528 * 373248
        assert algo < t < 2 * algo
