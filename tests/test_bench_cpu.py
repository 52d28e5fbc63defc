"""bench.py's host-side contract, without a GPU: the one-GPU guard and the
workload table (the sizes the JSON line names)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv, env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(argv, env):
    """Asked for more than one GPU (by flag or by a launcher's WORLD_SIZE),
    bench.py exits with status 2 and says why, before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                       env={**os.environ, **env}, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, (r.returncode, r.stderr)
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("key, name, nx, ny", [
    ("mach3", "mach3_reflection_2048x512", 2048, 512),
    ("bubble", "shock_bubble_4096x1024", 4096, 1024),
    ("couette", "couette_8192x2048", 8192, 2048),
    ("sod", "sod_400x4", 400, 4),
])
def test_workload_sizes_match_their_names(key, name, nx, ny):
    """Each single-grid workload builds the grid its name states; its crop
    (the oracle's sample) keeps the time step and node spacing."""
    w = bench.workloads()[key]
    assert w["name"] == name
    prob = w["make"]()
    assert (prob.nx, prob.ny) == (nx, ny)
    crop = w["crop"]()
    assert crop.dt == prob.dt and crop.dx == prob.dx
    assert crop.nx * crop.ny <= prob.nx * prob.ny


def test_roofline_constants():
    """128 B per node update (16 FP32 populations read and written once)
    against 8 TB/s; the VALU ceiling is the published FP32 vector rate over
    ~330 operations per node update."""
    assert bench.BYTES_PER_UPDATE == 16 * 4 * 2
    assert bench.HBM_PEAK_GBS == 8000.0
    assert abs(bench.ALU_NODE_RATE * 330 * 2 - 157.3e12) / 157.3e12 < 1e-3
