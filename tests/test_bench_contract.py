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
    # k_alpha: 19 populations of 2 components read in FP32, alpha * beta of
    # each component written in FP64, the type byte
    assert bench.alpha_bytes_per_node(4, 2) == 2 * 19 * 4 + 2 * 8 + 1 == 169
    # k_collide: populations read and written, alpha * beta read, psi of each
    # component, phi, |E|^2, q and the component densities (FP64 fields), type
    assert bench.collide_bytes_per_node(4, 8, 2) == 2 * 2 * 19 * 4 + 2 * 8 + 7 * 8 + 1 == 377
    assert bench.collide_bytes_per_node(4, 4, 2) == 304 + 16 + 28 + 1
    # whole step with k SOR sweeps
    assert bench.step_bytes_per_node(4, 2, 8) == 304 + 40 + 128


def test_ensemble_comparison_starts_where_the_autotuner_leaves_the_state():
    # the comparison starters run as many warm-up steps as the autotuner
    # advances the learned run: two rounds over each of its candidates of 32
    # steps, plus one graph replay before each trial (elbm_autotune)
    sys.path.insert(0, ROOT)
    import bench
    from paper_1612_05404_amd import elbm
    assert elbm.TUNE_CANDIDATES == 11
    graph_warmups = 2 * (4 + 2 + 2) * 2 + 2 * (2 + 4 + 8)
    assert bench.AUTOTUNE_STEPS == 2 * elbm.TUNE_CANDIDATES * 32 + graph_warmups == 764
