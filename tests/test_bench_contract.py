"""bench.py's host-side contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_node():
    sys.path.insert(0, ROOT)
    import bench
    # 19 populations of 2 components read and written in FP32, plus psi of each
    # component, phi, |E|^2, q, rho_A (FP32 field count) and the type byte
    assert bench.collide_bytes_per_node(4, 2) == 2 * 2 * 19 * 4 + 6 * 4 + 1 == 329
    assert bench.collide_bytes_per_node(8, 2) == 2 * 2 * 19 * 8 + 6 * 8 + 1
    # whole step with k SOR sweeps
    assert bench.step_bytes_per_node(4, 2, 8) == 304 + 40 + 128
