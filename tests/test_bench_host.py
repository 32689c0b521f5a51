"""Host-side checks of bench.py's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_covers_the_shared_filter_header():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.KERNEL_SOURCES["operators.hip"] == ("operators.hip", "filter.h")
    assert bench.KERNEL_SOURCES["aniso.hip"] == ("aniso.hip", "filter.h")
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash("operators.hip")
    assert h != bench.kernel_source_hash("aniso.hip")
