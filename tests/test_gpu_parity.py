"""GPU parity: the HIP step (through the C ABI) against the FP64 oracle on the
same seeded inputs, plus properties that hold at any size.

Tolerances (FP32 arithmetic against an FP64 reference):
* one step from arbitrary positive populations: |f_gpu - f_oracle| <=
  2e-6 max|f|.  A node's update is a chain of about 30 FP32 roundings
  (butterflies, 4x4 blocks, equilibria, back-map, stencil), each <= 2^-24 of
  a partial result no larger than a few max|f|: 30 * 6e-8 * ~1 ~ 2e-6.
* many steps of smooth flow: relative L1 <= 1e-5 on rho, u, p (the stated
  accuracy target for smooth flow).
* shocks: the density midpoint crossing within one cell of the oracle's.
* different kernel variants, graph replay, restart: bit for bit equal.
"""
import os

import numpy as np
import pytest

import synth
from oracle import core, metrics
from tests.rounding import equilibrium_scale, transform_scale

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
U32 = 2.0 ** -24  # FP32 unit roundoff
RATES = synth.rates(1e-5, s5=500, s6=700, s7=1000, s8=1100, s11=2500)
VARIANTS = [("simple", 0), ("rows", 1), ("rows", 2)]

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


def run_gpu(MRT2D, prob, f0=None, nsteps=1, **kw):
    g = MRT2D.from_problem(prob, **kw)
    if f0 is None:
        g.init_problem(prob)
    else:
        g.set_f(f0)
    g.step(nsteps)
    f = g.get_f_numpy()
    mac = g.macro_numpy()
    info = g.kernel_info()
    g.close()
    return f, mac, info


def run_oracle(prob, f0=None, nsteps=1):
    o = core.Grid(prob, nthreads=THREADS)
    if f0 is None:
        o.init_problem()
    else:
        o.set_f(f0)
    o.run(nsteps)
    return o.get_f(), o.macro()


@pytest.mark.parametrize("sides", sorted(SIDE_SETS))
def test_one_step_matches_oracle_every_variant(gpu, sides):
    """Arbitrary positive populations on a ragged 150x37 grid (several
    64-column strips plus a tail), one step, each boundary rule set, every
    kernel variant; and all variants agree bit for bit."""
    nx, ny = 150, 37
    f0 = synth.random_populations(nx, ny, seed=1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
    want, _ = run_oracle(prob, f0, 1)
    outs = []
    for kern, seg in VARIANTS:
        got, _, info = run_gpu(gpu, prob, f0, 1, kernel=kern, rows=seg)
        assert info == (kern, seg)
        err = np.max(np.abs(got - want))
        assert err <= 2e-6 * np.max(np.abs(want)), (kern, seg, err)
        outs.append(got)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("nx", [64, 128, 129, 193])
@pytest.mark.parametrize("sides", ["reflect_extrapolate", "wall_split", "dirichlet"])
def test_one_step_grid_widths(gpu, nx, sides):
    """Grid widths where the last column is lane 63 of its wave (64, 128), the
    only column of its wave (129) or lane 0 of a second wave past 128 (193),
    with odd and even heights: one step of every row-kernel variant matches
    the simple kernel bit for bit and the oracle within the one-step bound."""
    for ny in (5, 38):
        f0 = synth.random_populations(nx, ny, seed=nx + ny)
        prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
        want, _ = run_oracle(prob, f0, 1)
        ref, _, _ = run_gpu(gpu, prob, f0, 1, kernel="simple")
        assert np.max(np.abs(ref - want)) <= 2e-6 * np.max(np.abs(want))
        for kern, seg in VARIANTS[1:]:
            got, _, _ = run_gpu(gpu, prob, f0, 1, kernel=kern, rows=seg)
            assert np.array_equal(got, ref), (nx, ny, kern, seg, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("sides", ["reflect_extrapolate", "wall_split"])
def test_layouts_agree(gpu, sides):
    """The three device orders of f (population planes, interleaved rows,
    64-column tiles) give the same bits for every kernel variant over 20
    steps, and match the oracle."""
    nx, ny = 150, 37
    f0 = synth.random_populations(nx, ny, seed=17)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
    want, _ = run_oracle(prob, f0, 20)
    outs = []
    for layout in ("rows", "planes", "tiles"):
        for kern, seg in VARIANTS:
            outs.append(run_gpu(gpu, prob, f0, 20, kernel=kern, rows=seg, layout=layout)[0])
        outs.append(run_gpu(gpu, prob, f0, 20, layout=layout, graph_steps=4)[0])
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.max(np.abs(outs[0] - want)) <= 20 * 2e-6 * np.max(np.abs(want))


@pytest.mark.parametrize("shape", [(3, 3), (3, 70), (70, 3), (65, 4)])
@pytest.mark.parametrize("sides", sorted(SIDE_SETS))
def test_smallest_grids(gpu, shape, sides):
    """Degenerate shapes (3 x 3 is the smallest grid; one-wave and one-row-
    group grids; a width with a lone last column): five steps of every
    variant agree bit for bit and with the oracle."""
    nx, ny = shape
    f0 = synth.random_populations(nx, ny, seed=nx * 100 + ny)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
    want, _ = run_oracle(prob, f0, 5)
    outs = [run_gpu(gpu, prob, f0, 5, kernel=k, rows=r)[0] for k, r in VARIANTS]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.max(np.abs(outs[0] - want)) <= 5 * 2e-6 * np.max(np.abs(want))


def test_largest_grid_sampled(gpu):
    """A grid near the 4 GiB limit of one copy of f (8192 x 7990 nodes,
    32-bit buffer offsets up to 4.26e9 B), periodic on all four sides, one
    step of the row kernel with one and two rows per wave: sampled nodes --
    random ones, the last grid row and column, the corners -- agree with the
    oracle's node update computed from the same FP32 state.  The limit itself
    with wall sides: test_largest_grid_for_32bit_offsets."""
    nx, ny = 8192, 7990
    ic = synth.smooth_macro(nx, ny, seed=31, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"], ic)
    rng = np.random.default_rng(5)
    pts = [(int(i), int(j)) for i, j in zip(rng.integers(0, nx, 200), rng.integers(0, ny, 200))]
    pts += [(i, ny - 1) for i in (0, 1, 63, 64, nx - 65, nx - 2, nx - 1)]
    pts += [(nx - 1, j) for j in (0, 1, ny // 2, ny - 2)] + [(0, 0), (0, ny - 1)]
    for rows in (1, 2):
        g = gpu.from_problem(prob, kernel="rows", rows=rows)
        g.init_problem(prob)
        f0 = g.get_f_numpy()
        g.step(1)
        f1 = g.get_f_numpy()
        g.close()
        scale = float(np.max(np.abs(f0)))
        err = 0.0
        for i, j in pts:
            col = lambda a, b: f0[:, b % ny, a % nx]
            want = core.cell_update(prob, col(i, j), col(i + 1, j), col(i - 1, j), col(i, j + 1), col(i, j - 1))
            err = max(err, float(np.max(np.abs(f1[:, j, i] - want))))
        del f0, f1
        print(f"largest grid, rows {rows}: max err over {len(pts)} sampled nodes {err:.3e}")
        assert err <= 2e-6 * scale


@pytest.mark.parametrize("sides", ["periodic", "reflect_extrapolate", "wall_split"])
def test_smooth_flow_many_steps(gpu, sides):
    nx, ny = 130, 70
    ic = synth.smooth_macro(nx, ny, seed=3, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], ic)
    _, want = run_oracle(prob, None, 300)
    _, got, _ = run_gpu(gpu, prob, None, 300)
    for k in ("rho", "ux", "uy", "p"):
        assert metrics.rel_l1(got[k], want[k]) <= 1e-5, k


def test_sod_tube(gpu):
    """The Sod configuration (400x4, 10k steps to t = 0.2) in FP32 against the
    FP64 oracle: relative L1 <= 1e-5 on rho, u, p and the shock within one
    cell."""
    prob = synth.sod()
    _, want = run_oracle(prob, None, prob.nsteps)
    _, got, _ = run_gpu(gpu, prob, None, prob.nsteps)
    for k in ("rho", "ux", "p"):
        assert metrics.rel_l1(got[k], want[k]) <= 1e-5, (k, metrics.rel_l1(got[k], want[k]))
    x = prob.x_centres()
    lvl = 0.5 * (0.125 + 0.2043)
    a = metrics.crossing(x, want["rho"][1], lvl, lo=0.8)
    b = metrics.crossing(x, got["rho"][1], lvl, lo=0.8)
    assert abs(a - b) <= prob.dx


def test_uniform_flow_stays_bitwise_uniform(gpu):
    nx, ny = 100, 30
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"],
                         synth.uniform_ic(nx, ny, 1.3, 0.4, -0.2, 0.9))
    f, mac, _ = run_gpu(gpu, prob, None, 50)
    assert np.all(f == f[:, :1, :1])
    np.testing.assert_allclose(mac["rho"], 1.3, rtol=1e-6)
    np.testing.assert_allclose(mac["ux"], 0.4, rtol=1e-5)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_periodic_conservation_fp64_sums(gpu, precision):
    """On a periodic grid the FP64 totals of rho, j, e drift by FP32
    round-off only -- in the split-BF16x3 mode too, whose back-map has no
    columns for the conserved moments, as in FP32 (observed: 1e-8 .. 1e-7
    of the totals after 5000 steps in both modes)."""
    nx, ny = 200, 120
    ic = synth.smooth_macro(nx, ny, seed=9, du=0.3, dr=0.2)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"], ic)
    g = gpu.from_problem(prob, precision=precision)
    g.init_problem(prob)
    a = g.sums()
    g.step(1000)
    b = g.sums()
    g.close()
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    ref = o.sums()
    # FP64 sums of the FP32 state: the initial totals agree with the oracle
    # to FP32 rounding of the initial state, and drift by FP32 round-off only
    np.testing.assert_allclose(a, ref, rtol=1e-6, atol=1e-6 * abs(ref[0]))
    drift = np.abs(b - a) / np.array([a[0], a[0], a[0], a[3]])
    assert np.all(drift <= 2e-5), drift


def test_graph_replay_equals_direct_launches(gpu):
    nx, ny = 150, 37
    f0 = synth.random_populations(nx, ny, seed=4)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], None)
    direct, _, _ = run_gpu(gpu, prob, f0, 37, kernel="rows", rows=2)
    graph, _, _ = run_gpu(gpu, prob, f0, 37, kernel="rows", rows=2, graph_steps=8)
    assert np.array_equal(direct, graph)
    # replays after eager work in between
    g = gpu.from_problem(prob, kernel="rows", rows=2, graph_steps=4)
    g.set_f(f0)
    for n in (4, 9, 8, 16):
        g.step(n)
        g.sums()
    got = g.get_f_numpy()
    g.close()
    ref, _, _ = run_gpu(gpu, prob, f0, 37, kernel="simple")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("budget", [0, 1])
def test_every_graph_replay_matches_direct_launches(gpu, budget):
    """Each call replays the captured step graphs (8 steps per graph, the
    outflow budget's side-stream fork and join captured with them when on);
    between calls the program does its own eager work (FP64 sums, reading f,
    synchronisation).  After every call the state, the sums and the outflow
    totals equal those of a context that launches the same steps directly."""
    nx, ny = 150, 37
    f0 = synth.random_populations(nx, ny, seed=12)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], None)
    kw = dict(kernel="rows", rows=1, flux_budget=budget)
    g = gpu.from_problem(prob, graph_steps=8, **kw)
    d = gpu.from_problem(prob, graph_steps=0, **kw)
    g.set_f(f0)
    d.set_f(f0)
    for n in (8, 16, 3, 8, 24, 8):
        g.step(n)
        d.step(n)
        assert np.array_equal(g.get_f_numpy(), d.get_f_numpy()), n
        assert np.array_equal(np.array(g.sums()), np.array(d.sums())), n
        if budget:
            assert np.array_equal(np.array(g.outflow()), np.array(d.outflow())), n
    g.close()
    d.close()


@pytest.mark.parametrize("nx,ny", [(141, 43), (500, 40)])
def test_autotune_trial_steps_are_ordinary_steps(gpu, nx, ny):
    """The autotuner times the candidate kernels on steps of the run itself:
    a run that tunes (grid sizes unique to this test, so nothing is cached;
    500 columns make 8 tile columns, so both tile orders run) equals a run
    with a fixed kernel bit for bit, clock and time-dependent boundary split
    included, whether the first call is too short to tune or not; afterwards
    the choice is final and reported."""
    f0 = synth.random_populations(nx, ny, seed=6)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], None)
    ref, _, _ = run_gpu(gpu, prob, f0, 401, kernel="simple")
    g = gpu.from_problem(prob, graph_steps=16)
    g.set_f(f0)
    g.step(1)                      # too short to tune: default kernel
    assert g.kernel_details() == ("rows", 1, False)
    g.step(400)                    # tunes on its first steps
    kern, rows, streaming = g.kernel_details()
    step, _ = g.time()
    got = g.get_f_numpy()
    g.close()
    assert step == 401
    assert (kern, rows) in {("rows", 1), ("rows", 2), ("simple", 0)}
    assert np.array_equal(got, ref)
    # a second context of the same size takes the cached choice at once
    h = gpu.from_problem(prob)
    h.set_f(f0)
    h.step(1)
    assert h.kernel_details() == (kern, rows, streaming)
    h.close()


def test_graphs_captured_before_tuning_are_rebuilt(gpu):
    """A first call long enough to capture a step graph but too short to
    tune replays the default variant; the next, longer call tunes, and its
    replays (graphs rebuilt for the chosen variant) continue the same bits
    as a run that never uses graphs."""
    nx, ny = 331, 29
    f0 = synth.random_populations(nx, ny, seed=13)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["dirichlet"], None)
    ref, _, _ = run_gpu(gpu, prob, f0, 16 + 600, kernel="simple")
    g = gpu.from_problem(prob, graph_steps=16)
    g.set_f(f0)
    g.step(16)                     # one graph captured and replayed, no tuning
    assert g.kernel_details() == ("rows", 1, False)
    g.step(600)                    # tunes, then replays rebuilt graphs
    got = g.get_f_numpy()
    print("tuned", g.kernel_variant())
    g.close()
    assert np.array_equal(got, ref)


def test_bf16x3_autotune_variants_agree(gpu):
    """The split-BF16x3 step autotunes its store kind and tile order on steps
    of the run (a grid of 8 tile columns, so both orders run): the tuned run
    equals a run that never tunes (each call too short) bit for bit, and a
    second context takes the cached choice, which an FP32 context of the
    same size does not share."""
    nx, ny = 504, 36
    f0 = synth.random_populations(nx, ny, seed=8)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["reflect_extrapolate"], None)
    g = gpu.from_problem(prob, precision="bf16x3", graph_steps=0)
    g.set_f(f0)
    for _ in range(200):
        g.step(1)                  # each call too short to tune
    assert g.kernel_details() == ("mfma", 1, False)
    ref = g.get_f_numpy()
    g.close()
    t = gpu.from_problem(prob, precision="bf16x3", graph_steps=16)
    t.set_f(f0)
    t.step(200)                    # tunes on its first 4 x 34 steps
    tuned = t.kernel_details()
    got = t.get_f_numpy()
    t.close()
    print("bf16x3 tuned variant", tuned)
    assert tuned[0] == "mfma"
    assert np.array_equal(got, ref)
    h = gpu.from_problem(prob, precision="bf16x3")
    h.set_f(f0)
    h.step(1)
    assert h.kernel_details() == tuned
    h.close()
    k = gpu.from_problem(prob)
    k.set_f(f0)
    k.step(1)
    assert k.kernel_details()[0] == "rows"
    k.close()


@pytest.mark.parametrize("sides", sorted(SIDE_SETS))
def test_fused_budget_equals_side_stream_budget(gpu, sides):
    """The row kernel at one row per wave computes the outflow budget in
    leading blocks of its own grid; the simple kernel and the row kernel at
    two rows per wave get it from a separate kernel on a second stream.  Same state, same FP64 face sums in the same order: the outflow
    totals agree bit for bit after 50 steps (graph-replayed)."""
    nx, ny = 141, 43
    f0 = synth.random_populations(nx, ny, seed=14)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], None)
    out = {}
    for kernel, rows in (("simple", 0), ("rows", 1), ("rows", 2)):
        g = gpu.from_problem(prob, kernel=kernel, rows=rows, flux_budget=True, graph_steps=16)
        g.set_f(f0)
        g.step(50)
        out[(kernel, rows)] = (g.get_f_numpy(), np.array(g.outflow()))
        g.close()
    ref_f, ref_o = out[("simple", 0)]
    for key, (f, o) in out.items():
        assert np.array_equal(f, ref_f), key
        assert np.array_equal(o, ref_o), key


@pytest.mark.parametrize("sides", ["wall_split", "reflect_extrapolate", "periodic"])
def test_outflow_budget(gpu, sides):
    """Outflow budget (flux_budget): the GPU's FP64 outflow through each side
    matches the oracle's, periodic sides carry equal and opposite totals, the
    step results are unchanged by the budget, and the GPU's own FP64 sums
    close against its outflow up to the FP32 rounding of the updates."""
    nx, ny, n = 150, 37, 300
    ic = synth.smooth_macro(nx, ny, seed=12, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], ic)
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    o.run(n)
    g = gpu.from_problem(prob, flux_budget=True, graph_steps=16)
    g.init_problem(prob)
    s0 = g.sums()
    g.step(n)
    s1 = g.sums()
    out = g.outflow()
    f_budget = g.get_f_numpy()
    g.close()
    plain, _, _ = run_gpu(gpu, prob, None, n, graph_steps=16)
    assert np.array_equal(f_budget, plain)
    h = gpu.from_problem(prob, flux_budget=True, graph_steps=0)  # direct launches
    h.init_problem(prob)
    h.step(n)
    assert np.array_equal(h.outflow(), out)
    h.close()
    err = np.abs(out - o.outflow)
    tol = 1e-5 * (np.abs(o.outflow).sum() + 1e-3 * np.abs(s0).sum() / (nx * ny))
    print(f"{sides}: outflow\n{out}\nmax |gpu - oracle| {err.max():.3e} (tol {tol:.3e})")
    assert np.all(err <= tol)
    if sides == "periodic":
        assert np.array_equal(out[0], -out[1]) and np.array_equal(out[2], -out[3])
    resid = s1 - s0 + out.sum(axis=0)
    scale = np.abs(s0) + np.abs(s1) + np.abs(out).sum(axis=0)
    print(f"{sides}: GPU budget residual / scale {resid / scale}")
    assert np.all(np.abs(resid) <= 4 * n * U32 * scale)


def test_outflow_budget_bf16x3(gpu):
    """The matrix-core step with the outflow budget (fused into its grid or
    on the side stream, whichever the autotuned rows per wave allows): the
    step results are unchanged by the budget, graph replay and direct
    launches give the same totals, the totals close against the FP64 sums as
    in FP32, and they follow the oracle's outflow to the FP32 bound (the
    matrix-core back-map perturbs the populations by at most ~2^-15 of the
    collision increment)."""
    nx, ny, n = 150, 37, 300
    ic = synth.smooth_macro(nx, ny, seed=12, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], ic)
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    o.run(n)
    g = gpu.from_problem(prob, precision="bf16x3", flux_budget=True, graph_steps=16)
    g.init_problem(prob)
    s0 = g.sums()
    g.step(n)
    s1 = g.sums()
    out = g.outflow()
    f_budget = g.get_f_numpy()
    assert g.kernel_variant()[0] == "mfma"
    g.close()
    plain, _, _ = run_gpu(gpu, prob, None, n, graph_steps=16, precision="bf16x3")
    assert np.array_equal(f_budget, plain)
    h = gpu.from_problem(prob, precision="bf16x3", flux_budget=True, graph_steps=0)
    h.init_problem(prob)
    h.step(n)
    assert np.array_equal(h.outflow(), out)
    h.close()
    err = np.abs(out - o.outflow)
    tol = 1e-5 * (np.abs(o.outflow).sum() + 1e-3 * np.abs(s0).sum() / (nx * ny))
    print(f"bf16x3 outflow: max |gpu - oracle| {err.max():.3e} (tol {tol:.3e})")
    assert np.all(err <= tol)
    resid = s1 - s0 + out.sum(axis=0)
    scale = np.abs(s0) + np.abs(s1) + np.abs(out).sum(axis=0)
    print(f"bf16x3 budget residual / scale {resid / scale}")
    assert np.all(np.abs(resid) <= 4 * n * U32 * scale)


def test_restart_is_bitwise(gpu):
    """Checkpoint/restart: 2N steps equal N steps, get_f, a fresh context
    with set_f and the clock restored, N more steps -- bit for bit, with a
    time-dependent boundary rule in play."""
    nx, ny = 90, 40
    ic = synth.smooth_macro(nx, ny, seed=5)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["wall_split"], ic)
    full, _, _ = run_gpu(gpu, prob, None, 40)
    g = gpu.from_problem(prob)
    g.init_problem(prob)
    g.step(20)
    mid = g.get_f()
    step, t = g.time()
    g.close()
    assert step == 20 and abs(t - 20 * prob.dt) < 1e-15
    h = gpu.from_problem(prob)
    h.set_f(mid)
    h.set_step(step)
    h.step(20)
    again = h.get_f_numpy()
    h.close()
    assert np.array_equal(full, again)


def test_error_paths(gpu):
    from paper_0908_3749_amd import MrtfdError
    from paper_0908_3749_amd import _abi
    nx, ny = 40, 20
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"],
                         synth.uniform_ic(nx, ny, 1.0, 0.0, 0.0, 1.0))
    g = gpu.from_problem(prob)
    with pytest.raises(MrtfdError) as e:
        g.step(1)
    assert e.value.status == _abi.MRTFD_ERR_STATE
    bad = dict(prob.ic)
    bad["rho"] = prob.ic["rho"].copy()
    bad["rho"][3, 4] = -1.0
    g.init_macro(bad["rho"], bad["ux"], bad["uy"], bad["T"])
    with pytest.raises(MrtfdError) as e:
        g.sums()
    assert e.value.status == _abi.MRTFD_ERR_ARG
    g.init_problem(prob)
    g.sums()
    # zero steps change nothing; a negative count is rejected and leaves the
    # context usable
    f0 = g.get_f_numpy()
    clock = g.time()
    g.step(0)
    assert np.array_equal(g.get_f_numpy(), f0) and g.time() == clock
    with pytest.raises(MrtfdError) as e:
        g.step(-1)
    assert e.value.status == _abi.MRTFD_ERR_ARG
    g.step(2)
    assert g.time()[0] == clock[0] + 2
    f = g.get_f_numpy()
    f[2, 5, 5] = np.nan
    g.set_f(f)
    g.step(3)
    with pytest.raises(MrtfdError) as e:
        g.sums()
    assert e.value.status == _abi.MRTFD_ERR_NONFINITE
    g.close()




@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (0.125, 0.3, -0.2, 0.8),
                                   (2.4545, 2.177, -1.257, 4.753), (0.138, 0.0, 0.0, 7.246),
                                   (1.28, -0.377, 0.0, 1.29)])
def test_init_matches_oracle(gpu, state):
    """f = M^-1 f-hat^eq(rho, u, T) evaluated in FP32: each population within
    64 u of the magnitude sum_k |M^-1_ik| |f-hat^eq_k| that its evaluation
    cancels (FP32 unit roundoff u = 2^-24; 64 covers the ~20 roundings of the
    equilibria and the back-map)."""
    nx, ny = 70, 5
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"],
                         synth.uniform_ic(nx, ny, *state))
    g = gpu.from_problem(prob)
    g.init_problem(prob)
    got = g.get_f_numpy()[:, 0, 0]
    g.close()
    m = core.model()
    rho, ux, uy, T = state
    fh = core.feq_moments(rho, rho * ux, rho * uy, rho * (T + 0.5 * (ux * ux + uy * uy)))
    want = m.Minv @ fh
    scale = np.abs(m.Minv) @ np.abs(fh)
    ratio = np.abs(got - want) / (U32 * scale)
    print(f"init {state}: max err / (u scale) = {ratio.max():.2f}")
    assert np.all(ratio <= 64), ratio


def _steps_to_autotune(nx, ny):
    """Steps the library's first long-enough mrtfd_step call spends timing
    its candidates (rows per wave x store kind x tile order, plus the simple
    kernel; two passes), plus a few steps of the chosen variant."""
    cells = nx * ny
    reps = 2 * int(max(4.0, min(16.0, 3.4e7 / cells)))
    ncand = 9 if ((nx + 63) // 64) % 8 == 0 else 5
    return 2 * ncand * (reps + 2) + 4


def _full_size_start(prob, ref):
    """(stored FP32 start g0, f_ref per population, an oracle grid holding
    g0 + f_ref in FP64): the oracle's initial equilibrium, less f_ref when a
    reference state is set, rounded to FP32 as the library stores it."""
    from paper_0908_3749_amd import make_params, ref_populations
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    fr = np.zeros(16)
    if ref is not None:
        fr = ref_populations(make_params(prob.nx, prob.ny, prob.dx, prob.dy, prob.dt, prob.s, prob.sides,
                                         ref=ref))
    g0 = (o.get_f() - fr[:, None, None]).astype(np.float32)
    o.set_f(g0.astype(np.float64) + fr[:, None, None])
    return g0, fr, o


@pytest.mark.parametrize("config", ["mach3", "bubble", "couette"])
def test_full_size_steps_match_oracle(gpu, config):
    """At the benchmark's full sizes (2048x512 Mach reflection, 4096x1024
    shock-bubble, 8192x2048 Couette) and in its launch configuration (graph
    of 64 steps, the step kernel autotuned on the run's first steps, as
    bench.py runs it): enough steps from the oracle's initial state (rounded
    to FP32) for the autotuner to finish agree with the whole-grid FP64
    oracle node by node, within 4 n u S after n steps, S = transform_scale
    (each step's rounding is a few u of the magnitudes the collision
    cancels).  Couette runs stored relative to the gas at rest (1, 1), as
    bench.py runs it: the oracle starts from the GPU's stored values plus
    f_ref in FP64, and the GPU's result plus f_ref is compared."""
    prob = {"mach3": synth.mach_reflection, "bubble": synth.shock_bubble, "couette": synth.couette}[config]()
    ref = (1.0, 1.0) if config == "couette" else None
    n = _steps_to_autotune(prob.nx, prob.ny)
    g0, fr, o = _full_size_start(prob, ref)
    scale = transform_scale(prob, o.get_f())
    o.run(n)
    want = o.get_f()
    del o
    g = gpu.from_problem(prob, graph_steps=64, ref=ref)
    g.set_f(g0)
    del g0
    g.step(n)
    got = g.get_f_numpy()
    variant = g.kernel_variant()
    g.close()
    err = max(float(np.max(np.abs(got[q] + fr[q] - want[q]))) for q in range(16))
    bound = 4 * n * U32 * scale
    print(f"full size {config}, {n} steps, variant {variant}: max err {err:.3e}, bound {bound:.3e}")
    assert err <= bound


def test_full_size_bf16x3_couette_matches_oracle(gpu):
    """The mixed-precision workload at its full size (Couette 8192 x 2048,
    stored relative to (1, 1), the collision's blocks on the matrix cores)
    in bench.py's launch configuration (graph of 64 steps, rows per wave,
    store kind and tile order autotuned on the run's first steps): after the
    autotune's two passes it agrees with the whole-grid FP64 oracle node by
    node within n (2^-14 + 4 u) S, the one-step bound of the matrix-core
    products (test_bf16x3_one_step_error_bound) on top of the FP32 one per
    step, S = transform_scale."""
    prob = synth.couette()
    ref = (1.0, 1.0)
    cells = prob.nx * prob.ny
    reps = 2 * int(max(4.0, min(16.0, 3.4e7 / cells)))
    # rows per wave x store kind x tile order
    ncand = 8 if ((prob.nx + 63) // 64) % 8 == 0 else 4
    n = 2 * ncand * (reps + 2) + 4
    g0, fr, o = _full_size_start(prob, ref)
    scale = transform_scale(prob, o.get_f())
    o.run(n)
    want = o.get_f()
    del o
    g = gpu.from_problem(prob, graph_steps=64, precision="bf16x3", ref=ref)
    g.set_f(g0)
    del g0
    g.step(n)
    got = g.get_f_numpy()
    variant = g.kernel_variant()
    g.close()
    assert variant[0] == "mfma"
    err = max(float(np.max(np.abs(got[q] + fr[q] - want[q]))) for q in range(16))
    bound = n * (2.0 ** -14 + 4 * U32) * scale
    print(f"full size couette bf16x3, {n} steps, variant {variant}: max err {err:.3e}, bound {bound:.3e}")
    assert err <= bound


def test_full_size_fp64_couette_matches_oracle(gpu):
    """The FP64 form bench.py times beside the headline (Couette 8192 x 2048,
    stored relative to (1, 1) in FP64, graph of 64 steps, the step kernel
    autotuned on the run's first steps: one row per wave x store kind x
    tile order, plus the simple kernel): after the autotune's two passes it
    agrees with the whole-grid FP64 oracle node by node within n 16 u64 S
    (the FP64 one-step bound, test_gpu_fp64), S = transform_scale."""
    from paper_0908_3749_amd import make_params, ref_populations
    prob = synth.couette()
    ref = (1.0, 1.0)
    cells = prob.nx * prob.ny
    reps = 2 * int(max(4.0, min(16.0, 3.4e7 / cells)))
    ncand = 5 if ((prob.nx + 63) // 64) % 8 == 0 else 3
    n = 2 * ncand * (reps + 2) + 4
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    fr = ref_populations(make_params(prob.nx, prob.ny, prob.dx, prob.dy, prob.dt, prob.s, prob.sides, ref=ref))
    g0 = o.get_f() - fr[:, None, None]
    o.set_f(g0 + fr[:, None, None])
    scale = transform_scale(prob, o.get_f())
    o.run(n)
    want = o.get_f()
    del o
    g = gpu.from_problem(prob, graph_steps=64, precision="fp64", ref=ref)
    g.set_f64(g0)
    del g0
    g.step(n)
    got = g.get_f64_numpy()
    variant = g.kernel_variant()
    g.close()
    err = max(float(np.max(np.abs(got[q] + fr[q] - want[q]))) for q in range(16))
    bound = n * 16 * 2.0 ** -53 * scale
    print(f"full size couette fp64, {n} steps, variant {variant}: max err {err:.3e}, bound {bound:.3e}")
    assert err <= bound


def test_largest_grid_for_32bit_offsets(gpu):
    """Maximum size: 8192 x 8063 is the largest grid of that width whose copy
    of f (rows of 16 x 8320 floats and the padding ring) stays below 4 GiB,
    the range of the row kernels' 32-bit buffer offsets; one more row is
    refused at create.  The Couette set-up (periodic in x, walls south and
    north, so the last rows build wall ghosts at the largest offsets), two
    steps with one and with two rows per wave against the whole-grid FP64
    oracle, node by node within 4 n u S (S over a window of columns: the
    flow is uniform in x up to the 1e-3 velocity noise)."""
    nx, ny, n = 8192, 8063, 2
    prob = synth.couette(nx=nx, ny=ny)
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    f0 = o.get_f().astype(np.float32)
    o.set_f(f0.astype(np.float64))
    scale = transform_scale(prob, f0[:, :, :256].astype(np.float64))
    o.run(n)
    want = o.get_f()
    del o
    bound = 4 * n * U32 * scale
    for rows in (1, 2):
        g = gpu.from_problem(prob, kernel="rows", rows=rows, graph_steps=0)
        g.set_f(f0)
        g.step(n)
        got = g.get_f_numpy()
        variant = g.kernel_variant()
        g.close()
        err = max(float(np.max(np.abs(got[q] - want[q]))) for q in range(16))
        del got
        print(f"largest grid {nx}x{ny}, variant {variant}: max err {err:.3e}, bound {bound:.3e}")
        assert err <= bound


def _shock_x(prob, rho, row, lo, hi):
    x = prob.x_centres()
    r = rho[row]
    level = 0.5 * (np.max(r[(x >= lo) & (x <= hi)]) + np.min(r[(x >= lo) & (x <= hi)]))
    return metrics.crossing(x, r, level, lo=lo, hi=hi)


def test_mach_reflection_crop(gpu):
    """The 256x64 crop of the Mach-3 reflection (same dx, dt, rates and
    rules), compared after 1000 and 5000 steps.  Shock flow at T up to 4.75,
    where populations reach 20 and FP32 rounding of f alone is 1e-6 per
    step: relative L1 <= 1e-4, and the incident shock crossing every row
    within one cell of the oracle (at 1000 steps, while it is in the crop)."""
    prob = synth.mach_reflection(nx=256, ny=64, x0_cells=64)
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    g = gpu.from_problem(prob, graph_steps=64)
    g.init_problem(prob)
    done = 0
    for n in (1000, 5000):
        o.run(n - done)
        g.step(n - done)
        done = n
        want, got = o.macro(), g.macro_numpy()
        errs = {k: metrics.rel_l1(got[k], want[k]) for k in ("rho", "ux", "uy", "p")}
        print(f"mach3 crop {n} steps rel L1", errs)
        for k, v in errs.items():
            assert v <= 1e-4, (n, k, v)
        if n == 1000:
            for row in range(0, 64, 8):
                a = _shock_x(prob, want["rho"], row, 0.2, 0.77)
                b = _shock_x(prob, got["rho"], row, 0.2, 0.77)
                assert a is not None and abs(a - b) <= prob.dx, (row, a, b)
    g.close()


def test_shock_bubble_scaled(gpu):
    prob = synth.shock_bubble(nx=512, ny=128)
    _, want = run_oracle(prob, None, 300)
    _, got, _ = run_gpu(gpu, prob, None, 300)
    errs = {k: metrics.rel_l1(got[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    print("bubble 512x128 300 steps rel L1", errs)
    for k in ("rho", "p"):
        assert errs[k] <= 1e-5, (k, errs[k])


def test_couette_strip(gpu):
    """Couette strip (walls at rest and at U = 0.1, seeded 1e-3 noise),
    1000 steps: rho and p within 1e-5 relative L1 (smooth flow); u, whose
    noise part is 1e-3, within 1e-5 U node by node."""
    prob = synth.couette(nx=16, ny=256, noise=1e-3)
    _, want = run_oracle(prob, None, 1000)
    _, got, _ = run_gpu(gpu, prob, None, 1000)
    errs = {k: metrics.rel_l1(got[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    print("couette 16x256 1000 steps rel L1", errs, "u Linf", metrics.linf(got["ux"], want["ux"]))
    for k in ("rho", "p"):
        assert errs[k] <= 1e-5, (k, errs[k])
    # u = j / rho: j rounds by ~u sum_i |v_i f_i| ~ 2e-7 per step, and the
    # errors of 1000 steps add up like a random walk (~30x)
    assert metrics.linf(got["ux"], want["ux"]) <= 1e-5
    assert metrics.linf(got["uy"], want["uy"]) <= 1e-5


def test_bf16x3_one_step_error_bound(gpu):
    """Block products on the matrix cores: the forward blocks hold exact BF16
    weights against inputs split exactly into three BF16 parts, so the
    moments are FP32-accurate (tests/test_bf16_blocks_cpu.py).  The back-map
    holds its FP32 weights w exactly as three BF16 parts and splits its
    inputs x, the nonequilibrium moments d, into two (|x - hi - lo| <= 2^-17
    |x|); it leaves out the products of the weights' middle and low parts
    (<= 2^-8 |w|) with the inputs' low parts (<= 2^-8 |x|).  Per product that
    is at most (2^-16 + 2^-17) |w| |x|, so per population the collision errs
    by at most 1.5 2^-16 (|dt M^-1| |S| |d|)_i; with |d| <= |M f| + |M f^eq|,
    within twice the moment scale, the bound is 2^-14 (|dt M^-1| |S| |M|
    |f|)_i on top of the FP32 bound.  Every node runs the matrix-core
    products (the boundary waves too); the variants agree bit for bit."""
    nx, ny = 200, 40
    f0 = synth.random_populations(nx, ny, seed=8, spread=0.3)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS["periodic"], None)
    want, _ = run_oracle(prob, f0, 1)
    got, _, info = run_gpu(gpu, prob, f0, 1, precision="bf16x3")
    assert info[0] == "mfma"
    m = core.model()
    A = np.abs(m.Minv) * prob.dt @ np.diag(np.abs(RATES)) @ np.abs(m.M)
    scale = np.einsum("ik,kyx->iyx", A, np.abs(f0))
    bound = 2.0 ** -14 * scale + 2e-6 * np.max(np.abs(want))
    ratio = np.abs(got - want) / bound
    print(f"bf16x3 one step: max err {np.max(np.abs(got - want)):.3e}, max err/bound {ratio.max():.3f}")
    assert np.all(ratio <= 1.0)
    fp32, _, _ = run_gpu(gpu, prob, f0, 1)
    # the split products differ from the FP32 ones at nearly every node
    assert np.mean(np.any(got != fp32, axis=0)) > 0.9


def test_bf16x3_couette_strip(gpu):
    """Couette strip 256 x 256 (plainly stored populations, 500 steps): the
    matrix-core products add nothing visible to the FP32 step's error, which
    here comes from rounding the stored populations at the scale of |f| --
    relative L1 within 1.25 times FP32's on rho, u1 and p."""
    prob = synth.couette(nx=256, ny=256, noise=1e-3)
    _, want = run_oracle(prob, None, 500)
    _, got32, _ = run_gpu(gpu, prob, None, 500)
    _, got16, _ = run_gpu(gpu, prob, None, 500, precision="bf16x3")
    e32 = {k: metrics.rel_l1(got32[k], want[k]) for k in ("rho", "ux", "p")}
    e16 = {k: metrics.rel_l1(got16[k], want[k]) for k in ("rho", "ux", "p")}
    print("couette 256x256 500 steps rel L1: fp32", e32, "bf16x3", e16)
    for k in ("rho", "ux", "p"):
        assert e16[k] <= 1.25 * e32[k], (k, e16[k], e32[k])


def test_single_relaxation_time_mode(gpu):
    """S = I / tau (Sect. II): the single-relaxation-time mode is Eq. (3) with
    all rates equal -- bit for bit the MRT path with equal rates -- and it
    matches the oracle within the FP32 bounds (one step from arbitrary
    populations; 300 steps of smooth flow)."""
    nx, ny = 150, 37
    s_all = [0.0] * 4 + [1e5] * 12
    f0 = synth.random_populations(nx, ny, seed=21)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, s_all, SIDE_SETS["reflect_extrapolate"], None)
    want, _ = run_oracle(prob, f0, 1)
    srt, _, _ = run_gpu(gpu, prob, f0, 1, collision="srt")
    mrt, _, _ = run_gpu(gpu, prob, f0, 1, collision="mrt")
    assert np.array_equal(srt, mrt)
    assert np.max(np.abs(srt - want)) <= 2e-6 * np.max(np.abs(want))
    ic = synth.smooth_macro(nx, ny, seed=3, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, s_all, SIDE_SETS["periodic"], ic)
    _, want = run_oracle(prob, None, 300)
    _, got, _ = run_gpu(gpu, prob, None, 300, collision="srt")
    errs = {k: metrics.rel_l1(got[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    print("srt 300 steps rel L1", errs)
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)


def _tube_shock_cells(prob, rho_o, rho_g):
    """Offset in cells between the GPU's and the oracle's density midpoint
    crossings at each shock (between the star density and the far state)."""
    from oracle import riemann
    L, R = prob.meta["left"], prob.meta["right"]
    W = riemann.wave_speeds(L, R)
    x = prob.x_centres()
    J = prob.ny // 2
    t = prob.nsteps * prob.dt
    out = {}
    for side, far in (("left", L[0]), ("right", R[0])):
        if W[side + "_shock"]:
            xs = prob.meta["x0"] + W[side + "_head"] * t
            lvl = 0.5 * (W["rho_star_" + side] + far)
            a = metrics.crossing(x, rho_o[J], lvl, lo=xs - 0.1, hi=xs + 0.1)
            b = metrics.crossing(x, rho_g[J], lvl, lo=xs - 0.1, hi=xs + 0.1)
            assert a is not None and b is not None, (side, xs, a, b)
            out[side] = (a - b) / prob.dx
    return out


def _few_steps_within_rounding_bound(gpu, prob, n):
    """n steps from the oracle's initial state rounded to FP32: the GPU's f
    within 4 n u (S + E) of the FP64 oracle's, S = transform_scale, E =
    equilibrium_scale."""
    o = core.Grid(prob, nthreads=THREADS)
    o.init_problem()
    f0 = o.get_f().astype(np.float32)
    o.set_f(f0.astype(np.float64))
    scale = transform_scale(prob, o.get_f()) + equilibrium_scale(prob, o.get_f())
    o.run(n)
    got, _, _ = run_gpu(gpu, prob, f0, n)
    err = np.max(np.abs(got - o.get_f()))
    bound = 4 * n * U32 * scale
    print(f"{prob.name} {prob.nx}x{prob.ny}: {n} steps, max err {err:.3e}, bound {bound:.3e}, "
          f"(S + E) / max|f| = {scale / np.max(np.abs(f0)):.3g}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("name", ["two_shock", "colella"])
def test_paper_tubes(gpu, name):
    """The two-shock collision (Sect. V.A(d), 867 cells) and Colella's
    explosion wave (Sect. V.A(c), 4000 cells) at the paper's spacing: four
    steps from the same FP32 start agree with the FP64 oracle within the
    rounding bound.  Longer FP32 runs of these two do not follow the oracle:
    the populations of their hot states sum to 4e4 (two shocks) and 7e5
    (Colella, T = 1000) times rho, so every FP32 step rounds rho by 1e-3 to
    4e-2 of itself, the equilibria carry that into f (E is 4e4 and 7e5
    times max|f|), and a growing 1D mode of the two-shock west state (1.0026
    per step) amplifies the noise; only FP64 carries them."""
    prob = synth.two_shock() if name == "two_shock" else synth.colella()
    _few_steps_within_rounding_bound(gpu, prob, 4)


@pytest.mark.parametrize("name", ["regular_reflection", "mach15_crop", "heavy_bubble"])
def test_paper_2d_workloads(gpu, name):
    """Sect. V.B(a) regular reflection (300x100, Mach-5 inflow, full size),
    a 300x150 crop of the Sect. V.B(b) Mach-1.5 reflection (same dx, dt,
    rates and rules, wedge from cell 75), and the Sect. V.C heavy bubble at
    512x128.  Four steps within the rounding bound; then FP32 against FP64
    after 2000 steps (300 for the bubble): relative L1 <= 1e-4 on rho, u1,
    u2, p for the Mach-1.5 crop (as for the Mach-3 crop), <= 1e-5 on rho,
    u1, p for the bubble (its u2 is a near-zero field: mean |du2| <= 1e-5
    max |u|), and for the regular reflection <= 2e-3 on rho and p with the
    incident and reflected shocks within one cell of the oracle's on every
    tenth column: its Mach-5 inflow has E ~ 400 max|f| (FP32 rounds f by
    ~4e-6 max|f| per step, against ~1e-8 in the Mach-1.5 flow) and a
    transverse mode growing by 1.0012 per step, so the per-step noise grows
    to ~1e-3 in the shocked flow by 1000 steps."""
    if name == "regular_reflection":
        prob, n = synth.regular_reflection(), 2000
    elif name == "mach15_crop":
        prob, n = synth.paper_mach_reflection(nx=300, ny=150), 2000
    else:
        prob, n = synth.heavy_bubble(nx=512, ny=128), 300
    _few_steps_within_rounding_bound(gpu, prob, 4)
    _, want = run_oracle(prob, None, n)
    _, got, _ = run_gpu(gpu, prob, None, n)
    errs = {k: metrics.rel_l1(got[k], want[k]) for k in ("rho", "ux", "uy", "p")}
    print(f"{name} {prob.nx}x{prob.ny} {n} steps rel L1 {errs}")
    if name == "mach15_crop":
        for k, v in errs.items():
            assert v <= 1e-4, (k, v)
    elif name == "heavy_bubble":
        for k in ("rho", "ux", "p"):
            assert errs[k] <= 1e-5, (k, errs[k])
        umax = np.max(np.hypot(want["ux"], want["uy"]))
        assert np.mean(np.abs(got["uy"] - want["uy"])) <= 1e-5 * umax
    else:
        for k in ("rho", "p"):
            assert errs[k] <= 2e-3, (k, errs[k])
        y = prob.y_centres()
        for i in range(5, prob.nx, 10):
            col_o, col_g = want["rho"][:, i], got["rho"][:, i]
            lvl = 0.5 * (np.max(col_o) + np.min(col_o))
            a = metrics.crossing(y, col_o, lvl)
            b = metrics.crossing(y, col_g, lvl)
            assert (a is None) == (b is None), (i, a, b)
            if a is not None:
                assert abs(a - b) <= prob.dy, (i, a, b)


@pytest.mark.parametrize("sides", sorted(SIDE_SETS))
def test_padding_is_never_read(gpu, sides, monkeypatch):
    """Both copies of f start as NaN outside the interior
    (MRTFD_POISON_PADDING=1): after 20 steps on a ragged grid (the last tile
    column is mostly padding) every kernel variant, the split-BF16x3 one
    included, gives the same bits as with zeroed padding, all finite -- no
    kernel reads a node outside the interior as state."""
    nx, ny = 141, 43
    ic = synth.smooth_macro(nx, ny, seed=11, du=0.2, dr=0.1)
    prob = synth.generic(nx, ny, 2e-3, 1e-5, RATES, SIDE_SETS[sides], ic)
    for kernel, rows, prec in [(k, r, "fp32") for k, r in VARIANTS] + [("auto", 0, "bf16x3")]:
        kw = dict(kernel=kernel, rows=rows, precision=prec)
        monkeypatch.delenv("MRTFD_POISON_PADDING", raising=False)
        clean, _, _ = run_gpu(gpu, prob, None, 20, **kw)
        monkeypatch.setenv("MRTFD_POISON_PADDING", "1")
        poisoned, _, info = run_gpu(gpu, prob, None, 20, **kw)
        monkeypatch.delenv("MRTFD_POISON_PADDING")
        assert np.all(np.isfinite(poisoned)), (info, prec)
        assert np.array_equal(poisoned, clean), (info, prec)
