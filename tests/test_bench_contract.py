"""Host-side checks of bench.py's contract (no GPU): the multi-GPU request is
refused with a message, and the committed counter summary of the streaming
apply matches the kernel source it was taken on (else the bench line's
traffic field would silently read null)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "single MI355X" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_matches_the_kernel_source():
    import bench
    t = bench.measured_traffic("dense8192")
    assert t is not None, "profiles/apply_stream_kernel.dense8192.traffic.md was taken on another apply.hip"
    assert 5.0e8 < t < 7.0e8
    assert bench.measured_traffic("casida262144") is None
