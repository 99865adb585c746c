"""Host-side checks of the benchmark's contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The benchmark measures one GPU; --gpus above 1 exits with a message and no JSON line."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert "{" not in r.stdout


def test_source_hash_covers_the_kernel_sources():
    """The traffic records are used only while the kernel sources hash to their recorded value."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    rec = bench.read_traffic("dst_cols", "2d_m255_n256", 6)
    assert rec is None or rec > 0
