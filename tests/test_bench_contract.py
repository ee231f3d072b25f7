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


def test_fused_launch_counts_one_read_of_x():
    """Per sweep of an order-3 tensor: the mode-0 launch carrying the X step
    moves read + mask + unobserved writes, modes 1 and 2 one read each."""
    sys.path.insert(0, ROOT)
    import bench
    nX, rd, upd = bench.algorithmic_bytes((256, 256, 31), 4, 0.1)
    assert bench.contraction_bytes(300, 99, rd, upd) == 201 * rd + 99 * upd
    assert bench.contraction_bytes(3, 1, rd, upd) == 2 * rd + upd
    assert bench.contraction_bytes(3, 0, rd, upd) == 3 * rd
