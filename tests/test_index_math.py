"""The node-index arithmetic every kernel uses (neighbour index with periodic
wrap, the index division by a box extent), compiled for the host from the
library's own header and checked against a direct definition."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_neighbour_index_and_extent_division(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "index_math")
    src = os.path.join(ROOT, "tests", "native", "index_math.hip")
    subprocess.run([hipcc, "-O1", "-std=c++17", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
                    "-o", exe, src], check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches 0" in r.stdout
