"""bench.py's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_formula():
    sys.path.insert(0, ROOT)
    import bench
    nX, rd, upd = bench.algorithmic_bytes((256, 256, 31), 4, 0.1)
    assert nX == 2031616
    assert rd == 4 * nX
    assert abs(upd - nX * (4 + 0.125 + 0.9 * 4)) < 1e-6
