"""Host-side logic of bench.py (no GPU): the one-GPU refusal and the key
that ties recorded profiler counters to the step kernel's sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_source_key_is_stable_and_records_are_consistent():
    sys.path.insert(0, ROOT)
    import bench
    key = bench.kernel_source_hash()
    assert len(key) == 16 and key == bench.kernel_source_hash()
    # both records are keyed the same way, and the recorded HBM traffic is
    # at least the algorithmic bytes of a launch
    assert bench.TRAFFIC["src"] == bench.VALU["src"]
    assert bench.TRAFFIC["bytes_per_launch"] >= bench.BYTES_PER_CELL_FP64 * bench.NX * bench.NY


def test_external_library_gets_no_recorded_counters(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setenv("SVE_LIBRARY", "/nonexistent/libsve.so")
    assert bench.kernel_source_hash() == "external"
