"""bench.py refuses more than one GPU before touching any device (CPU only)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields():
    """The oracle leg of the bench line (CPU only): a bounded sample, its
    rate, and the cores it used."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench.cpu_baseline(0.3, threads=1)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "expansions/s"
    assert r["value"] > 0 and "partial 8-tree" in r["sample"]
