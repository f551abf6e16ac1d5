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


def test_traffic_summaries_exist_and_match_their_kernel_source():
    """Every workload with a counter summary names the source it was taken on;
    the summary is used only while that source is unchanged, and then holds a
    plausible per-launch figure (between the algorithmic bytes and 1.5x)."""
    import hashlib
    import bench
    t = bench.measured_traffic("dense8192")
    assert t is not None, "profiles/apply_stream_kernel.dense8192.traffic.md was taken on another apply.hip"
    assert 5.41e8 <= t < 1.5 * 5.41e8
    for workload, (fname, src, key) in bench.TRAFFIC.items():
        with open(os.path.join(ROOT, "profiles", fname)) as fh:
            text = fh.read()
        assert key + ":" in text and "traffic_bytes_per_launch:" in text, fname
        with open(os.path.join(bench.CSRC, src), "rb") as fh:
            same = hashlib.sha256(fh.read()).hexdigest() in text
        assert (bench.measured_traffic(workload) is not None) == same, workload
    assert bench.measured_traffic("dense32768") is None
