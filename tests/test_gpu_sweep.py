"""A seeded sweep of random configurations through the C ABI against the FP64
oracle.  Each case draws a grid size (inside one tile, ragged, several
tiles), a boundary rule per side (periodic pairs, Dirichlet, reflecting,
extrapolating, walls, and two-rule sides whose switch point moves by a few
cells over the run), random rates s5..s16, a reference state or none, FP32,
the matrix-core collision or FP64, a kernel variant and a population layout, and
starts from random populations or from smooth macroscopic fields.  The
oracle starts from the GPU's own initial state (the stored values plus
f_ref, in FP64) and both run n steps; every population must agree within
n (8 u + c) S, S = transform_scale of the initial state, c = 0 in FP32 and
2^-14 with the matrix cores (their one-step bound,
test_gpu_parity.test_bf16x3_one_step_error_bound); in FP64, n 16 u64 S."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import core
from tests.rounding import transform_scale

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
U32 = 2.0 ** -24
DX, DT = 2e-3, 1e-5
KINDS = ["dirichlet", "reflect", "extrapolate", "wall"]
NCASES = 64


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3749_amd import MRT2D
    torch.cuda.set_device(0)
    return MRT2D


def draw(seed):
    rng = np.random.default_rng(seed)
    nx = int(rng.choice([3, 5, 17, 63, 64, 65, 127, 129, 200, 257]))
    ny = int(rng.choice([3, 4, 7, 33, 64, 65, 130]))
    nsteps = int(rng.choice([1, 3]))

    def state():
        return (float(rng.uniform(0.5, 2.0)), float(rng.uniform(-0.3, 0.3)),
                float(rng.uniform(-0.3, 0.3)), float(rng.uniform(0.5, 2.0)))

    sides = {}
    for a, b, length in (("west", "east", ny * DX), ("south", "north", nx * DX)):
        if rng.random() < 0.35:
            sides[a] = sides[b] = synth.side("periodic")
            continue
        for sd in (a, b):
            if rng.random() < 0.3:
                k1, k2 = (str(k) for k in rng.choice(KINDS, 2))
                # the switch point moves by up to 3 cells over the run
                rate = float(rng.uniform(-3.0, 3.0)) * DX / (nsteps * DT)
                sides[sd] = synth.split_side(k1, state(), k2, state(), float(rng.uniform(0.0, length)), rate)
            else:
                sides[sd] = synth.side(str(rng.choice(KINDS)), state())
    s = [0.0] * 4 + [float(v) for v in np.exp(rng.uniform(math.log(100.0), math.log(1.0 / DT), 12))]
    precision = "bf16x3" if rng.random() < 0.3 else "fp32"
    if precision == "fp32":
        kernel, rows = [("simple", 0), ("rows", 1), ("rows", 2), ("auto", 0)][int(rng.integers(4))]
    else:
        kernel, rows = "auto", 0
    case = dict(nx=nx, ny=ny, nsteps=nsteps, sides=sides, s=s, precision=precision, kernel=kernel, rows=rows,
                layout=str(rng.choice(["rows", "tiles", "planes"])),
                ref=(float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.5, 2.0))) if rng.random() < 0.5 else None,
                init="populations" if rng.random() < 0.5 else "macro", seed=int(seed))
    if precision == "fp32" and rng.random() < 0.3:  # drawn last: the other choices stay as they were
        case["precision"] = "fp64"
        if case["kernel"] == "rows":
            case["kernel"], case["rows"] = "auto", 0
    return case


def describe(c):
    sd = {k: (v["kind_lo"] if v["kind_lo"] == v["kind_hi"] else f"{v['kind_lo']}|{v['kind_hi']}")
          for k, v in c["sides"].items()}
    return (f"seed {c['seed']}: {c['nx']}x{c['ny']}, {c['nsteps']} steps, {c['precision']}, "
            f"{c['kernel']}/{c['rows']}, layout {c['layout']}, ref {c['ref']}, init {c['init']}, sides {sd}")


@pytest.mark.parametrize("seed", range(1000, 1000 + NCASES))
def test_random_configuration_matches_oracle(gpu, seed):
    from paper_0908_3749_amd import make_params, ref_populations

    c = draw(seed)
    print(describe(c), flush=True)
    nx, ny = c["nx"], c["ny"]
    ic = synth.smooth_macro(nx, ny, seed=seed, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, DX, DT, c["s"], c["sides"], ic)
    fr = np.zeros(16)
    if c["ref"] is not None:
        fr = ref_populations(make_params(nx, ny, DX, DX, DT, c["s"], c["sides"], ref=c["ref"]))
    g = gpu.from_problem(prob, precision=c["precision"], kernel=c["kernel"], rows=c["rows"],
                         layout=c["layout"], ref=c["ref"])
    if c["init"] == "populations":
        f0 = synth.random_populations(nx, ny, seed=seed, spread=0.3)
        g.set_f64(f0 - fr[:, None, None])
    else:
        g.init_problem(prob)
    start = g.get_f64_numpy() + fr[:, None, None]
    g.step(c["nsteps"])
    got = g.get_f64_numpy() + fr[:, None, None]
    g.close()
    o = core.Grid(prob, nthreads=THREADS)
    o.set_f(start)
    o.run(c["nsteps"])
    want = o.get_f()
    assert np.all(np.isfinite(got))
    S = transform_scale(prob, start)
    if c["precision"] == "fp64":
        bound = c["nsteps"] * 16 * 2.0 ** -53 * S
    else:
        extra = 2.0 ** -14 if c["precision"] == "bf16x3" else 0.0
        bound = c["nsteps"] * (8 * U32 + extra) * S
    err = float(np.max(np.abs(got - want)))
    print(f"  max err {err:.3e}, bound {bound:.3e} ({err / bound:.3f})", flush=True)
    assert err <= bound
