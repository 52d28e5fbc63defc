"""Pins of the oracle's space-time scheme and boundary rules: the Fourier
amplification of the Lax-Wendroff/Euler update, uniform flow, global
conservation on periodic grids, translation, mirror and rotation symmetry,
and the ghost-node states of every boundary rule."""
import math

import numpy as np
import pytest

import synth
from oracle import analytic, core

PER = {k: synth.side("periodic") for k in synth.SIDES}


def periodic_problem(nx, ny, s, dx=0.01, dt=2e-4, ic=None):
    if ic is None:
        ic = synth.uniform_ic(nx, ny, 1.0, 0.0, 0.0, 1.0)
    return synth.generic(nx, ny, dx, dt, s, dict(PER), ic)


@pytest.mark.parametrize("kx,ky", [(1, 0), (0, 2), (3, 1), (2, 5)])
def test_fourier_mode_amplification(kx, ky):
    """With all rates zero the update is pure advection of each population;
    one Fourier mode is multiplied by 1 - i c_x sin(th_x) + c_x^2 (cos th_x - 1)
    - i c_y sin(th_y) + c_y^2 (cos th_y - 1) per step (Sect. IV, the
    advective part of G)."""
    nx, ny, dx, dt = 16, 12, 0.01, 4e-4
    prob = periodic_problem(nx, ny, [0.0] * 16, dx=dx, dt=dt)
    g = core.Grid(prob)
    m = core.model()
    rng = np.random.default_rng(kx * 10 + ky)
    A = rng.normal(size=16) + 1j * rng.normal(size=16)
    bg = core.feq_velocity(1.0, 0.0, 0.0, 1.0)
    x = np.arange(nx)
    y = np.arange(ny)
    thx, thy = 2 * math.pi * kx / nx, 2 * math.pi * ky / ny
    phase = np.exp(1j * (thx * x[None, :] + thy * y[:, None]))
    amp = 0.1
    f0 = bg[:, None, None] + amp * np.real(A[:, None, None] * phase[None])
    g.set_f(f0)
    g.run(1)
    got = g.get_f() - bg[:, None, None]
    for i in range(16):
        G = analytic.lw_amplification(m.v[i, 0] * dt / dx, m.v[i, 1] * dt / dx, thx, thy)
        expect = amp * np.real(A[i] * G * phase)
        assert np.max(np.abs(got[i] - expect)) <= 1e-13, i


def test_uniform_flow_stays_uniform_periodic():
    nx, ny = 7, 5
    state = (1.3, 0.4, -0.2, 0.9)
    s = synth.rates(1e-4, s5=500, s6=700, s7=900, s8=1100)
    prob = periodic_problem(nx, ny, s, dx=0.01, dt=1e-4, ic=synth.uniform_ic(nx, ny, *state))
    g = core.Grid(prob)
    g.init_problem()
    f0 = g.get_f().copy()
    g.run(20)
    f = g.get_f()
    # every cell identical, bit for bit
    assert np.all(f == f[:, :1, :1])
    assert np.max(np.abs(f - f0)) <= 1e-13 * np.max(np.abs(f0))


@pytest.mark.parametrize("kind", ["dirichlet", "reflect", "extrapolate", "wall"])
def test_uniform_flow_with_open_boundaries(kind):
    """A uniform state parallel to the x walls is kept by every rule when the
    boundary state equals it (wall/reflect need uy = 0 at the y sides)."""
    nx, ny = 6, 5
    state = (0.9, 0.35, 0.0, 1.2)
    s = synth.rates(1e-4, s5=2000, s7=3000)
    sides = {"west": synth.side("periodic"), "east": synth.side("periodic"),
             "south": synth.side(kind, state), "north": synth.side(kind, state)}
    if kind == "dirichlet":
        state = (0.9, 0.35, -0.1, 1.2)
        sides = {k: synth.side("dirichlet", state) for k in synth.SIDES}
    prob = synth.generic(nx, ny, 0.01, 1e-4, s, sides, synth.uniform_ic(nx, ny, *state))
    g = core.Grid(prob)
    g.init_problem()
    f0 = g.get_f().copy()
    g.run(10)
    assert np.max(np.abs(g.get_f() - f0)) <= 1e-13 * np.max(np.abs(f0))


def test_periodic_totals_conserved():
    nx, ny = 24, 20
    ic = synth.smooth_macro(nx, ny, seed=3, du=0.3, dr=0.2)
    s = synth.rates(5e-5, s5=800, s6=900, s7=1200, s8=1500, s11=2500)
    prob = periodic_problem(nx, ny, s, dx=0.01, dt=5e-5, ic=ic)
    g = core.Grid(prob)
    g.init_problem()
    a = g.sums()
    g.run(40)
    b = g.sums()
    scale = np.array([abs(a[0]), abs(a[0]), abs(a[0]), abs(a[3])])
    assert np.all(np.abs(b - a) <= 1e-12 * scale)
    # and the run really moved mass around
    assert np.max(np.abs(g.macro()["rho"] - ic["rho"])) > 1e-4


def test_translation_invariance_bitwise():
    nx, ny = 11, 9
    ic = synth.smooth_macro(nx, ny, seed=5)
    s = synth.rates(1e-4, s5=1000, s7=2000)
    prob = periodic_problem(nx, ny, s, dx=0.01, dt=1e-4)
    f0 = synth.random_populations(nx, ny, seed=1)
    a = core.Grid(prob)
    a.set_f(f0)
    a.run(5)
    b = core.Grid(prob)
    b.set_f(np.roll(f0, (2, 3), axis=(1, 2)))
    b.run(5)
    assert np.array_equal(np.roll(a.get_f(), (2, 3), axis=(1, 2)), b.get_f())
    assert ic["rho"].shape == (ny, nx)


def _perm(transform):
    v = core.model().v
    out = []
    for i in range(16):
        w = transform(v[i])
        j = int(np.argmin(np.hypot(*(v - w).T)))
        assert np.hypot(*(v[j] - w)) < 1e-12
        out.append(j)
    return np.array(out)


def test_mirror_symmetry_in_x():
    """Mirroring x (and swapping the populations with opposite v_x) commutes
    with the update, for any rates."""
    nx, ny = 10, 6
    s = synth.rates(1e-4, s5=1000, s6=1500, s7=2000, s8=2500, s9=3000, s10=3500,
                    s11=4000, s13=4500, s14=5000, s15=5500, s16=6000)
    prob = periodic_problem(nx, ny, s, dx=0.01, dt=1e-4)
    perm = _perm(lambda w: np.array([-w[0], w[1]]))
    f0 = synth.random_populations(nx, ny, seed=11)
    a = core.Grid(prob)
    a.set_f(f0)
    a.run(3)
    fm = np.empty_like(f0)
    fm[perm] = f0[:, :, ::-1]
    b = core.Grid(prob)
    b.set_f(fm)
    b.run(3)
    want = np.empty_like(f0)
    want[perm] = a.get_f()[:, :, ::-1]
    assert np.max(np.abs(b.get_f() - want)) <= 1e-13 * np.max(np.abs(want))


def test_rotation_symmetry():
    """A quarter turn commutes with the update when s7 = s8, s9 = s10 and
    s15 = s16 (rates of moments that a quarter turn mixes)."""
    n = 8
    s = synth.rates(1e-4, s5=1000, s6=1500, s7=2000, s8=2000, s9=3000, s10=3000,
                    s11=4000, s13=4500, s14=5000, s15=5500, s16=5500)
    prob = periodic_problem(n, n, s, dx=0.01, dt=1e-4)
    perm = _perm(lambda w: np.array([-w[1], w[0]]))  # (vx, vy) -> (-vy, vx)
    f0 = synth.random_populations(n, n, seed=12)

    def rot(f):  # field rotated by +90 degrees: new[j][i] = old[i][n-1-j] ... as arrays
        out = np.empty_like(f)
        out[perm] = np.rot90(f, k=1, axes=(2, 1))
        return out

    a = core.Grid(prob)
    a.set_f(f0)
    a.run(3)
    b = core.Grid(prob)
    b.set_f(rot(f0))
    b.run(3)
    want = rot(a.get_f())
    assert np.max(np.abs(b.get_f() - want)) <= 1e-12 * np.max(np.abs(want))


def test_rotation_symmetry_breaks_with_unequal_rates():
    n = 8
    s = synth.rates(1e-4, s5=1000, s7=2000, s8=9000)
    prob = periodic_problem(n, n, s, dx=0.01, dt=1e-4)
    perm = _perm(lambda w: np.array([-w[1], w[0]]))
    f0 = synth.random_populations(n, n, seed=12)

    def rot(f):
        out = np.empty_like(f)
        out[perm] = np.rot90(f, k=1, axes=(2, 1))
        return out

    a = core.Grid(prob)
    a.set_f(f0)
    a.run(3)
    b = core.Grid(prob)
    b.set_f(rot(f0))
    b.run(3)
    assert np.max(np.abs(b.get_f() - rot(a.get_f()))) > 1e-8


# ------------------------------------------------------------ boundary rules

def ghost_macro(g, side, a):
    """(rho, u1, u2, T, p) of ghost node number a on a side."""
    f = g.f
    if side == "west":
        node = f[a + 1, 0]
    elif side == "east":
        node = f[a + 1, -1]
    elif side == "south":
        node = f[0, a + 1]
    else:
        node = f[-1, a + 1]
    return core.macro_of(node)


def linear_ic(nx, ny, dx):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    return {"rho": 1.0 + 2.0 * X + 1.0 * Y, "ux": 0.3 - 1.5 * X + 0.5 * Y,
            "uy": -0.2 + 0.7 * X - 2.0 * Y, "T": 1.0 + 0.5 * X + 3.0 * Y}


def lin(x, y):
    return np.array([1.0 + 2.0 * x + 1.0 * y, 0.3 - 1.5 * x + 0.5 * y,
                     -0.2 + 0.7 * x - 2.0 * y, 1.0 + 0.5 * x + 3.0 * y])


def test_extrapolation_ghosts_are_linear_extrapolation():
    nx, ny, dx = 6, 5, 0.05
    sides = {k: synth.side("extrapolate") for k in synth.SIDES}
    prob = synth.generic(nx, ny, dx, 1e-4, synth.rates(), sides, linear_ic(nx, ny, dx))
    g = core.Grid(prob)
    g.init_problem()
    for a in range(ny):
        y = (a + 0.5) * dx
        np.testing.assert_allclose(ghost_macro(g, "west", a)[:4], lin(-0.5 * dx, y), rtol=1e-12)
        np.testing.assert_allclose(ghost_macro(g, "east", a)[:4], lin((nx + 0.5) * dx, y), rtol=1e-12)
    for a in range(nx):
        x = (a + 0.5) * dx
        np.testing.assert_allclose(ghost_macro(g, "south", a)[:4], lin(x, -0.5 * dx), rtol=1e-12)
        np.testing.assert_allclose(ghost_macro(g, "north", a)[:4], lin(x, (ny + 0.5) * dx), rtol=1e-12)


def test_extrapolation_falls_back_to_nearest_state():
    nx, ny, dx = 5, 4, 1.0
    ic = synth.uniform_ic(nx, ny, 1.0, 0.0, 0.0, 1.0)
    ic["rho"][:, 0] = 0.2   # 2*0.2 - 1.0 < 0
    sides = {k: synth.side("extrapolate") for k in synth.SIDES}
    prob = synth.generic(nx, ny, dx, 1e-4, synth.rates(), sides, ic)
    g = core.Grid(prob)
    g.init_problem()
    np.testing.assert_allclose(ghost_macro(g, "west", 1)[:4], [0.2, 0.0, 0.0, 1.0], atol=1e-14)


def test_reflect_wall_dirichlet_periodic_ghosts():
    nx, ny, dx = 6, 5, 0.05
    ic = linear_ic(nx, ny, dx)
    wall = (7.0, 0.25, -0.05, 1.5)
    dstate = (0.8, 0.1, 0.2, 0.6)
    sides = {"west": synth.side("reflect"), "east": synth.side("dirichlet", dstate),
             "south": synth.side("wall", wall), "north": synth.side("periodic")}
    prob = synth.generic(nx, ny, dx, 1e-4, synth.rates(), sides, ic)
    g = core.Grid(prob)
    g.init_problem()
    for a in range(ny):
        y = (a + 0.5) * dx
        q1 = lin(0.5 * dx, y)
        np.testing.assert_allclose(ghost_macro(g, "west", a)[:4], [q1[0], -q1[1], q1[2], q1[3]], rtol=1e-12)
        np.testing.assert_allclose(ghost_macro(g, "east", a)[:4], dstate, rtol=1e-12, atol=1e-14)
    for a in range(nx):
        x = (a + 0.5) * dx
        q1 = lin(x, 0.5 * dx)
        np.testing.assert_allclose(ghost_macro(g, "south", a)[:4], [q1[0], wall[1], wall[2], wall[3]],
                                   rtol=1e-12)
        # periodic: north ghost is a copy of the bottom interior row
        assert np.array_equal(g.f[-1, a + 1], g.f[1, a + 1])


def test_split_side_moves_with_time():
    """kind_lo applies where the along-side coordinate <= split0 + rate t."""
    nx, ny, dx, dt = 10, 3, 0.1, 0.01
    post = (2.0, 0.5, 0.0, 1.5)
    sides = {"west": synth.side("periodic"), "east": synth.side("periodic"),
             "south": synth.side("periodic"),
             "north": synth.split_side("dirichlet", post, "extrapolate", (1, 0, 0, 1), 0.32, 10.0)}
    prob = synth.generic(nx, ny, dx, dt, synth.rates(dt), sides, synth.uniform_ic(nx, ny, 1.0, 0.0, 0.0, 1.0))
    g = core.Grid(prob)
    g.init_problem()            # t = 0: split at 0.32 -> nodes x = 0.05..0.25 post
    rho = [ghost_macro(g, "north", a)[0] for a in range(nx)]
    np.testing.assert_allclose(rho, [2.0] * 3 + [1.0] * 7, rtol=1e-12)
    g.run(3)                    # t = 0.03: split at 0.62 -> x = 0.05..0.55 post
    rho = [ghost_macro(g, "north", a)[0] for a in range(nx)]
    np.testing.assert_allclose(rho[:6], [2.0] * 6, rtol=1e-12)
    assert all(abs(r - 2.0) > 0.1 for r in rho[6:])


# ---------------------------------------------------------------- outflow budget

def test_outflow_of_a_uniform_state_is_the_euler_flux():
    """Uniform state with every side held at that state: nothing changes, and
    the outflow per step through a side is the Euler flux of the state times
    the side's node count times dt/h -- rho u_n, rho u u_n + P n, (e + P) u_n
    -- with the sign of the outward normal (closed forms of the equilibrium's
    moments, Eq. 14)."""
    nx, ny, dx, dt = 12, 10, 0.01, 2e-4
    rho, ux, uy, T = 1.3, 0.4, -0.2, 0.9
    st = (rho, ux, uy, T)
    sides = {k: synth.side("dirichlet", st) for k in synth.SIDES}
    prob = synth.generic(nx, ny, dx, dt, synth.rates(dt, s5=300.0), sides,
                         synth.uniform_ic(nx, ny, *st))
    g = core.Grid(prob)
    g.init_problem()
    g.run(1)
    P = rho * T
    e = rho * (T + 0.5 * (ux * ux + uy * uy))
    flux_x = np.array([rho * ux, rho * ux * ux + P, rho * ux * uy, (e + P) * ux])
    flux_y = np.array([rho * uy, rho * ux * uy, rho * uy * uy + P, (e + P) * uy])
    c = dt / dx
    np.testing.assert_allclose(g.outflow[1], ny * c * flux_x, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(g.outflow[0], -ny * c * flux_x, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(g.outflow[3], nx * c * flux_y, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(g.outflow[2], -nx * c * flux_y, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("which", ["sod", "mach3_crop", "mixed_rules"])
def test_outflow_budget_closes(which):
    """Over the interior, the sums of rho, j, e change by minus the outflow
    through the sides (the A.1b difference in flux form; the collision
    conserves them): closes to FP64 round-off on open boundaries of every
    kind, over many steps and time-dependent rule switches."""
    if which == "sod":
        prob = synth.sod(nx=200)
        n = 400
    elif which == "mach3_crop":
        prob = synth.mach_reflection(nx=96, ny=32, x0_cells=24)
        n = 300
    else:
        nx, ny = 40, 30
        sides = {"west": synth.side("extrapolate"), "east": synth.side("wall", (1.0, 0.0, 0.3, 1.2)),
                 "south": synth.split_side("dirichlet", (1.5, 0.2, 0.1, 1.1), "reflect",
                                           (1.0, 0.0, 0.0, 1.0), 0.1, 3.0),
                 "north": synth.side("extrapolate")}
        ic = synth.smooth_macro(nx, ny, seed=9, du=0.3, dr=0.2)
        prob = synth.generic(nx, ny, 0.01, 1e-4, synth.rates(1e-4, s5=800.0, s7=2e3), sides, ic)
        n = 300
    g = core.Grid(prob)
    g.init_problem()
    s0 = g.sums()
    g.run(n)
    s1 = g.sums()
    out = g.outflow.sum(axis=0)
    scale = np.abs(s0) + np.abs(s1) + np.abs(g.outflow).sum(axis=0) + 1.0
    resid = (s1 - s0 + out) / scale
    print(which, "budget residual", resid, "outflow", out)
    assert np.all(np.abs(resid) <= 1e-12), resid
    assert np.any(np.abs(out) > 1e-6 * scale)  # the sides do carry flux


def test_periodic_sides_have_no_net_outflow():
    nx, ny = 24, 16
    ic = synth.smooth_macro(nx, ny, seed=4)
    prob = periodic_problem(nx, ny, synth.rates(2e-4, s5=500.0), ic=ic)
    g = core.Grid(prob)
    g.init_problem()
    g.run(50)
    np.testing.assert_array_equal(g.outflow[0], -g.outflow[1])
    np.testing.assert_array_equal(g.outflow[2], -g.outflow[3])
