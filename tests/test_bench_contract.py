"""bench.py's fixed parts, on the CPU: the algorithmic bytes per lattice
update that its roofline figures use, and the refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bytes_per_lup():
    """2 (N - 1 + nc + Q) s: the state read once and written once, phi counted
    N - 1 times, U derived."""
    import bench
    from paper_2608_26908_amd.workloads import workload
    assert bench.bytes_per_lup(workload("dendrite3d"), 4) == 168
    assert bench.bytes_per_lup(workload("dendrite3d"), 8) == 336
    assert bench.bytes_per_lup(workload("dendrite3d", lattice="D3Q27"), 4) == 232
    assert bench.bytes_per_lup(workload("eutectic4_3d"), 4) == 192
    assert bench.bytes_per_lup(workload("eutectic2d"), 4) == 96
    assert bench.bytes_per_lup(workload("dendrite2d"), 8) == 176


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""

