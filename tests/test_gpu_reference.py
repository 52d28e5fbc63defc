"""GPU parity of the reference-state storage: with a reference state at rest
(rho0, T0) the library stores g = f - f_ref, f_ref = f^eq(rho0, 0, 0, T0)
(Eq. 14 mapped back by M^-1).  The difference scheme (Eq. A.1b) is linear and
f_ref uniform, so it acts on g alone; the collision (Eq. 3) adds back the
reference's conserved moments.  These tests compare g + f_ref (FP64) with the
FP64 oracle's f on the same inputs:

* one step from arbitrary populations: within the FP32 one-step bound
  2e-6 max|f| for every kernel variant (and the variants bit for bit);
* the reference state itself is an exact fixed point (g stays 0 bit for bit,
  wall ghosts at the reference included);
* smooth flow near the reference: the Couette strip after 2000 steps within
  relative L1 1e-5 on rho, u and p;
* restart, FP64 sums and the outflow budget with the reference's share
  added back.
"""
import os

import numpy as np
import pytest

import synth
from oracle import core, metrics

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
U32 = 2.0 ** -24
RATES = synth.rates(1e-5, s5=500, s6=700, s7=1000, s8=1100, s11=2500)
REF = (1.0, 1.0)

SIDE_SETS = {
    "periodic": {k: synth.side("periodic") for k in synth.SIDES},
    "dirichlet": {"west": synth.side("dirichlet", (1.0, 0.1, 0.0, 1.0)),
                  "east": synth.side("dirichlet", (0.5, 0.0, 0.1, 0.8)),
                  "south": synth.side("periodic"), "north": synth.side("periodic")},
    "reflect_extrapolate": {"west": synth.side("extrapolate"), "east": synth.side("extrapolate"),
                            "south": synth.side("reflect"), "north": synth.side("reflect")},
    "wall_split": {"west": synth.side("periodic"), "east": synth.side("periodic"),
                   "south": synth.side("wall", (1.0, 0.0, 0.0, 1.0)),
                   "north": synth.split_side("dirichlet", (2.0, 0.3, -0.2, 1.5), "extrapolate",
                                             (1.0, 0.0, 0.0, 1.0), 0.2, 5.0)},
}


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_3749_amd import MRT2D
    torch.cuda.set_device(0)
    return MRT2D


def f_ref(prob, ref=REF):
    from paper_0908_3749_amd import make_params, ref_populations
    p = make_params(prob.nx, prob.ny, prob.dx, prob.dy, prob.dt, prob.s, prob.sides, ref=ref)
    return ref_populations(p)


def oracle_run(prob, f0, n):
    o = core.Grid(prob, nthreads=THREADS)
    if f0 is None:
        o.init_problem()
    else:
        o.set_f(f0)
    o.run(n)
    return o


@pytest.mark.parametrize("sides", sorted(SIDE_SETS))
def test_one_step_every_variant(gpu, sides):
    """Arbitrary positive populations on a ragged 150x37 grid, one step: the
    stored g of every kernel variant plus f_ref within 2e-6 max|f| of the
    oracle, and the variants bit for bit."""
    nx, ny = 150, 37
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
    fr = f_ref(prob)[:, None, None]
    f0 = synth.random_populations(nx, ny, seed=31)
    g0 = (f0 - fr).astype(np.float32)
    want = oracle_run(prob, g0.astype(np.float64) + fr, 1).get_f()
    outs = []
    for kern, rows in (("simple", 0), ("rows", 1), ("rows", 2)):
        g = gpu.from_problem(prob, kernel=kern, rows=rows, ref=REF)
        g.set_f(g0)
        g.step(1)
        got = g.get_f_numpy()
        g.close()
        err = np.max(np.abs(got.astype(np.float64) + fr - want))
        print(f"{sides} {kern}/{rows}: max err {err:.3e}, bound {2e-6 * np.max(np.abs(want)):.3e}")
        assert err <= 2e-6 * np.max(np.abs(want)), (kern, rows, err)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_one_step_bf16x3(gpu):
    """The matrix-core block products on stored deviations: every node within
    the bound 2^-14 (|dt M^-1| |S| |M| |g|)_i of the back-map's split inputs
    (test_gpu_parity.test_bf16x3_one_step_error_bound; the transforms act on
    g here) on top of the FP32 one, and different from the FP32 step."""
    nx, ny = 200, 40
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"], None)
    fr = f_ref(prob)[:, None, None]
    f0 = synth.random_populations(nx, ny, seed=8, spread=0.3)
    g0 = (f0 - fr).astype(np.float32)
    want = oracle_run(prob, g0.astype(np.float64) + fr, 1).get_f()
    g = gpu.from_problem(prob, precision="bf16x3", ref=REF)
    g.set_f(g0)
    g.step(1)
    got = g.get_f_numpy()
    assert g.kernel_variant()[0] == "mfma"
    g.close()
    h = gpu.from_problem(prob, ref=REF)
    h.set_f(g0)
    h.step(1)
    fp32 = h.get_f_numpy()
    h.close()
    m = core.model()
    A = np.abs(m.Minv) * prob.dt @ np.diag(np.abs(RATES)) @ np.abs(m.M)
    scale = np.einsum("ik,kyx->iyx", A, np.abs(g0.astype(np.float64)))
    bound = 2.0 ** -14 * scale + 2e-6 * np.max(np.abs(want))
    err = np.abs(got.astype(np.float64) + fr - want)
    print(f"bf16x3 with reference: max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.mean(np.any(got != fp32, axis=0)) > 0.9


@pytest.mark.parametrize("sides", ["periodic", "wall_rest"])
def test_reference_state_is_a_fixed_point(gpu, sides):
    """Gas at rest in the reference state (rho0, T0): the stored g is zero at
    init and stays zero bit for bit over 200 steps, for every kernel variant
    (walls at rest at T0 build zero ghosts)."""
    nx, ny = 150, 37
    sd = SIDE_SETS["periodic"] if sides == "periodic" else {
        "west": synth.side("periodic"), "east": synth.side("periodic"),
        "south": synth.side("wall", (1.0, 0.0, 0.0, 1.0)),
        "north": synth.side("wall", (1.0, 0.0, 0.0, 1.0))}
    ic = synth.uniform_ic(nx, ny, REF[0], 0.0, 0.0, REF[1])
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, sd, ic)
    for kern, rows in (("simple", 0), ("rows", 1), ("rows", 2)):
        g = gpu.from_problem(prob, kernel=kern, rows=rows, ref=REF)
        g.init_problem(prob)
        assert not np.any(g.get_f_numpy())
        g.step(200)
        assert not np.any(g.get_f_numpy()), (kern, rows)
        mac = g.macro_numpy()
        g.close()
        assert np.all(mac["rho"] == 1.0) and np.all(mac["T"] == 1.0) and not np.any(mac["ux"])


def _couette_errors(gpu, prob, n, **kw):
    g = gpu.from_problem(prob, graph_steps=64, **kw)
    g.init_problem(prob)
    g.step(n)
    got = g.macro_numpy()
    g.close()
    return got


def test_couette_strip_within_smooth_flow_target(gpu):
    """Couette strip 16x256 (walls at rest and at U = 0.1, 1e-3 seeded noise),
    2000 steps: with the reference state (1, 1) the FP32 step stays within
    relative L1 1e-5 of the FP64 oracle on rho, u and p (the smooth-flow
    target), and its u error is below the plain FP32 storage's."""
    prob = synth.couette(nx=16, ny=256, noise=1e-3)
    want = oracle_run(prob, None, 2000).macro()
    shifted = _couette_errors(gpu, prob, 2000, ref=REF)
    plain = _couette_errors(gpu, prob, 2000)
    e_s = {k: metrics.rel_l1(shifted[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    e_p = {k: metrics.rel_l1(plain[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    print("couette 16x256 2000 steps rel L1: reference", e_s, "plain", e_p)
    for k in ("rho", "ux", "p"):
        assert e_s[k] <= 1e-5, (k, e_s[k])
    assert e_s["ux"] < e_p["ux"]


def test_restart_is_bitwise(gpu):
    nx, ny = 90, 40
    ic = synth.smooth_macro(nx, ny, seed=5)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], ic)
    g = gpu.from_problem(prob, ref=REF)
    g.init_problem(prob)
    g.step(40)
    full = g.get_f_numpy()
    g.close()
    g = gpu.from_problem(prob, ref=REF)
    g.init_problem(prob)
    g.step(20)
    mid = g.get_f()
    step, _ = g.time()
    g.close()
    h = gpu.from_problem(prob, ref=REF)
    h.set_f(mid)
    h.set_step(step)
    h.step(20)
    again = h.get_f_numpy()
    h.close()
    assert np.array_equal(full, again)


@pytest.mark.parametrize("sides", ["wall_split", "dirichlet"])
def test_sums_and_outflow_budget(gpu, sides):
    """FP64 sums and the outflow budget with the reference's share added back
    on the host: sums match the oracle's, the outflow matches the oracle's
    within 1e-5 of the total, and the budget closes against the sums."""
    nx, ny, n = 150, 37, 300
    ic = synth.smooth_macro(nx, ny, seed=12, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], ic)
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    so = o.sums()
    o.run(n)
    g = gpu.from_problem(prob, flux_budget=True, graph_steps=16, ref=REF)
    g.init_problem(prob)
    s0 = g.sums()
    g.step(n)
    s1 = g.sums()
    out = g.outflow()
    g.close()
    assert np.all(np.abs(s0 - so) <= 1e-6 * np.abs(so).sum())
    assert np.all(np.abs(s1 - o.sums()) <= 1e-5 * np.abs(so).sum())
    err = np.abs(out - o.outflow)
    tol = 1e-5 * (np.abs(o.outflow).sum() + 1e-3 * np.abs(s0).sum() / (nx * ny))
    print(f"{sides}: outflow max |gpu - oracle| {err.max():.3e} (tol {tol:.3e})")
    assert np.all(err <= tol)
    resid = s1 - s0 + out.sum(axis=0)
    scale = np.abs(s0) + np.abs(s1) + np.abs(out).sum(axis=0)
    print(f"{sides}: GPU budget residual / scale {resid / scale}")
    assert np.all(np.abs(resid) <= 4 * n * U32 * scale)
