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
    against 8 TB/s; the VALU ceiling is half the published FP32 vector rate
    (157.3 TFLOP/s counts packed FP32, two lanes of work per instruction,
    which the library's build leaves out), i.e. 64 lane-operations per CU
    and clock, over ~330 operations per node update: 119 G node updates/s."""
    assert bench.BYTES_PER_UPDATE == 16 * 4 * 2
    assert bench.HBM_PEAK_GBS == 8000.0
    assert abs(bench.ALU_NODE_RATE * 330 * 2 * 2 - 157.3e12) / 157.3e12 < 1e-3
    assert abs(bench.ALU_NODE_RATE - 119.2e9) < 0.1e9


def test_default_workload_is_the_hbm_resident_couette():
    """With no flags, bench.py times the Couette flow on 8192 x 2048 nodes
    (2 x 1 GiB of populations, beyond the 256 MB last-level cache), stored
    as deviations from the equilibrium at rest of rho = T = 1."""
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--config", default="couette"' in src
    w = bench.workloads()["couette"]
    assert w["ref"] == (1.0, 1.0) and w["steps"] == 50000
    prob = w["make"]()
    assert 2 * 16 * 4 * prob.nx * prob.ny >= 2 * 2 ** 30


def test_host_threads():
    threads, nproc, avail = bench.host_threads()
    assert 1 <= threads <= avail <= nproc


def test_input_riemann_solver_matches_the_oracles():
    """The input generators' own exact Riemann solver (used to size the tube
    runs without touching the oracle) agrees with the oracle's on random
    states of the batch's ranges, both gammas, and reports vacuum alike; the
    default batch is the same whichever builds it."""
    import numpy as np

    import synth
    from oracle import riemann

    rng = np.random.default_rng(3)
    for gamma in (2.0, 1.4):
        for _ in range(500):
            L = (rng.uniform(0.1, 5), rng.uniform(-2, 2), rng.uniform(0.1, 100))
            R = (rng.uniform(0.1, 5), rng.uniform(-2, 2), rng.uniform(0.1, 100))
            if riemann.has_vacuum(L, R, gamma):
                with pytest.raises(ValueError):
                    synth.riemann_waves(L, R, gamma)
                continue
            a, b = synth.riemann_waves(L, R, gamma), riemann.wave_speeds(L, R, gamma)
            for k in ("pstar", "ustar", "rho_star_left", "rho_star_right", "left_head", "left_tail",
                      "right_head", "right_tail"):
                assert abs(a[k] - b[k]) <= 1e-12 * max(1.0, abs(b[k])), (k, a[k], b[k])
            assert (a["left_shock"], a["right_shock"]) == (b["left_shock"], b["right_shock"])

    def oracle_star(L, R):
        W = riemann.wave_speeds(L, R)
        rmin = min(W["rho_star_left"], W["rho_star_right"])
        return riemann.max_signal_speed(L, R), rmin, W["pstar"] / rmin

    assert synth.tube_batch(star_fn=synth.tube_star) == synth.tube_batch(star_fn=oracle_star)
