"""bench.py on the host: more than one GPU is refused with a message; the roofline's operation
and byte models give the counts stated with the bench lines."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unsplit_reading_is_refused_for_event_workloads():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "ensemble",
                        "--unsplit-hancock"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "hotspot and shock" in r.stderr
    assert r.stdout == ""


def test_roofline_models():
    sys.path.insert(0, ROOT)
    import bench
    # p = e/3, MC, k = 3: reconstruction 4 x (2 + 5 + 2), Hancock 2 x 22 + 16, MUSTA 3 (66 + 44) + 2 x 24,
    # difference 8
    assert bench.flops_per_cell_axis(3, 3) == 482
    # the ideal gas with the charge, minmod, k = 4, five components
    assert bench.C2P_FLUX_GAS == 31 and bench.NEWTON_ITER_FLOPS_GAS == 24
    fx = bench.flops_per_cell_axis(4, 1, bench.C2P_FLUX_GAS, nc=5)
    assert fx == 804
    # y and z: 13 of the 14 solves per cell skip the residual at p = 0 (18) and the start (1)
    assert bench.GAS_WARM_SKIP == 19
    assert abs(bench.gas_flops_per_cell_axis(4, 1) - (804 + 2 * (804 - 13 * 19)) / 3) < 1e-9
    # algorithmic HBM bytes per cell-step: RK2 5 passes, RK3 8, of nc components
    assert bench.bytes_per_cell_step(2, 8) == 160
    assert bench.bytes_per_cell_step(3, 8, 5) == 320

