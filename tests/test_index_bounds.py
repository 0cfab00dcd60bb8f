"""Host check that the sweeps' index maps stay inside their arrays.

Compiles tests/index_bounds.cpp (plain g++, no GPU) against the kernels' own
index header and runs it: every load, look-ahead and store index of the y/z
march, the x sweep's row stream and the unsplit pre-pass, for lines of 1..9
cells (and longer rows), both boundary rules and many segment lengths, lies in
its array, and each sweep writes every cell exactly once.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sweep_indices_stay_in_bounds(tmp_path):
    exe = str(tmp_path / "index_bounds")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1510_06340_amd", "csrc"),
                    os.path.join(ROOT, "tests", "index_bounds.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok ")
