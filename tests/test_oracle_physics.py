"""Pins of the whole oracle against physics the paper fixes: shock tubes
against the exact Riemann solution (gamma = 2), a shear wave and Couette flow
against the discretisation-corrected viscosity, plus self-checks of the
reference solutions and of the seeded shock states."""
import math

import numpy as np
import pytest

import synth
from oracle import analytic, core, metrics, riemann
from tests.golden import parse


# ------------------------------------------------- reference-solution checks

def test_exact_solver_textbook_gamma_1_4():
    """Sod's problem at gamma = 1.4: p* = 0.30313, u* = 0.92745 (Toro,
    Riemann Solvers and Numerical Methods for Fluid Dynamics, Table 4.2)."""
    p, u = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma=1.4)
    assert abs(p - 0.30313) < 5e-6 and abs(u - 0.92745) < 5e-6


def _conserved(rho, u, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * u * u
    return np.array([rho, rho * u, E]), np.array([rho * u, rho * u * u + p, u * (E + p)])


@pytest.mark.parametrize("gamma", [2.0, 1.4])
@pytest.mark.parametrize("L,R", [((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
                                 ((5.99924, 19.5975, 460.894), (5.99242, -6.19633, 46.0950)),
                                 ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571))])
def test_exact_solution_satisfies_jump_conditions(L, R, gamma):
    """Across each shock S [U] = [F(U)]; across each fan the entropy p/rho^g
    and the outgoing Riemann invariant are constant; p and u are continuous
    at the contact."""
    W = riemann.wave_speeds(L, R, gamma)
    eps = 1e-9
    for side in ("left", "right"):
        head, tail = W[side + "_head"], W[side + "_tail"]
        if W[side + "_shock"]:
            a = riemann.sample(L, R, [head - eps, head + eps], gamma)
            U1, F1 = _conserved(a[0][0], a[1][0], a[2][0], gamma)
            U2, F2 = _conserved(a[0][1], a[1][1], a[2][1], gamma)
            np.testing.assert_allclose(head * (U2 - U1), F2 - F1, rtol=1e-9, atol=1e-9)
        else:
            xs = np.linspace(min(head, tail), max(head, tail), 7)
            r, u, p = riemann.sample(L, R, xs, gamma)
            ent = p / r ** gamma
            np.testing.assert_allclose(ent, ent[0], rtol=1e-10)
            a = np.sqrt(gamma * p / r)
            inv = u + 2 * a / (gamma - 1) if side == "left" else u - 2 * a / (gamma - 1)
            np.testing.assert_allclose(inv, inv[0], rtol=1e-10, atol=1e-10)
    c = W["contact"]
    r, u, p = riemann.sample(L, R, [c - eps, c + eps], gamma)
    np.testing.assert_allclose(p[0], p[1], rtol=1e-7)
    np.testing.assert_allclose(u[0], u[1], rtol=1e-7, atol=1e-9)


def test_paper_shock_states_are_gamma_2():
    """The post-shock states printed in Sect. V.B(b) and V.C follow the
    Rankine-Hugoniot relations of a gamma = 2 gas, not of gamma = 1.4."""
    for label, (rho1, p1, mach, rho2, u2, p2) in parse.paper_states().items():
        r, u, p, _ = synth.normal_shock(rho1, p1, mach, gamma=2.0)
        np.testing.assert_allclose([r, u, p], [rho2, u2, p2], rtol=2e-4, err_msg=label)
        r14, _, p14, _ = synth.normal_shock(rho1, p1, mach, gamma=1.4)
        assert abs(r14 - rho2) / rho2 > 0.05 or abs(p14 - p2) / p2 > 0.03, label


def test_paper_mach_numbers_are_gamma_2():
    """Sect. V.A(e): 'Mach number of the left side is 10.1, and the right is
    6.3' for (u, T) = (45, 10) and (-20, 5): |u| / sqrt(gamma T) with gamma = 2."""
    assert round(45.0 / math.sqrt(2.0 * 10.0), 1) == 10.1
    assert round(20.0 / math.sqrt(2.0 * 5.0), 1) == 6.3
    assert round(45.0 / math.sqrt(1.4 * 10.0), 1) != 10.1


def test_couette_series():
    U, D, nu = 0.1, 0.132, 2e-3
    y = np.linspace(0.0, D, 41)
    # boundary values for all t, rest at t = 0 (Gibbs aside), linear when steady
    for t in (0.0, 0.5, 3.0):
        u = analytic.couette_one_wall(y, t, U, D, nu)
        assert abs(u[0]) < 1e-12 and abs(u[-1] - U) < 1e-12
    assert np.max(np.abs(analytic.couette_one_wall(y[5:-5], 0.0, U, D, nu, nterms=20000))) < 2e-3
    np.testing.assert_allclose(analytic.couette_one_wall(y, 1e4, U, D, nu), U * y / D, atol=1e-12)
    # the diffusion equation u_t = nu u_yy holds
    t, h, k = 0.3, 1e-4, 1e-3
    yy = np.linspace(0.02, D - 0.02, 9)
    ut = (analytic.couette_one_wall(yy, t + k, U, D, nu) - analytic.couette_one_wall(yy, t - k, U, D, nu)) / (2 * k)
    uyy = (analytic.couette_one_wall(yy + h, t, U, D, nu) - 2 * analytic.couette_one_wall(yy, t, U, D, nu)
           + analytic.couette_one_wall(yy - h, t, U, D, nu)) / h ** 2
    np.testing.assert_allclose(ut, nu * uyy, rtol=2e-3, atol=1e-6)
    # the paper's two-wall form: odd in y, +-U at the walls
    yp = np.linspace(-D / 2, D / 2, 21)
    up = analytic.couette_paper(yp, 0.2, U, D, nu)
    np.testing.assert_allclose(up, -up[::-1], atol=1e-14)
    assert abs(up[-1] - U) < 1e-12


# ---------------------------------------------------------- whole-scheme pins

def _tube_errors(prob, grid, left, right):
    mac = grid.macro()
    x = prob.x_centres()
    r, u, p, T = riemann.profile(left, right, x, prob.meta["x0"], grid.t, 2.0)
    J = prob.ny // 2
    return {k: metrics.paper_error(mac[k][J], ex)
            for k, ex in (("rho", r), ("ux", u), ("p", p), ("T", T))}, mac, x


@pytest.mark.slow
def test_sod_matches_exact_solution():
    prob = synth.sod()
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    E, mac, x = _tube_errors(prob, g, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert E["rho"] < 0.03 and E["p"] < 0.03 and E["ux"] < 0.05 and E["T"] < 0.04, E
    W = riemann.wave_speeds((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    xs = 0.5 + W["right_head"] * g.t
    level = 0.5 * (W["rho_star_right"] + 0.125)
    pos = metrics.crossing(x, mac["rho"][1], level, lo=xs - 0.1, hi=xs + 0.1)
    assert abs(pos - xs) <= prob.dx, (pos, xs)
    # y-uniformity of a 1D problem is exact
    assert np.all(mac["rho"] == mac["rho"][:1])


@pytest.mark.slow
def test_lax_matches_exact_solution():
    prob = synth.lax()
    L, R = prob.meta["left"], prob.meta["right"]
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    E, mac, x = _tube_errors(prob, g, L, R)
    assert E["rho"] < 0.04 and E["p"] < 0.03 and E["ux"] < 0.05 and E["T"] < 0.04, E
    W = riemann.wave_speeds(L, R)
    xs = prob.meta["x0"] + W["right_head"] * g.t
    level = 0.5 * (W["rho_star_right"] + R[0])
    pos = metrics.crossing(x, mac["rho"][1], level, lo=xs - 0.1, hi=xs + 0.1)
    assert abs(pos - xs) <= 2 * prob.dx, (pos, xs)


@pytest.mark.slow
def test_shear_wave_decays_with_corrected_viscosity():
    """u1 = A sin(k y) decays as exp(-nu' k^2 t) with nu' = T (1/s6 + dt/2)
    (the discretisation-corrected shear viscosity of the appendix), and not
    with the uncorrected T / s6."""
    s6, dt = 2000.0, 1e-4
    prob = synth.shear_wave(nx=4, ny=64, dx=1.0 / 256, dt=dt, amp=1e-3, s_shear=s6, nsteps=8000)
    g = core.Grid(prob, nthreads=4)
    g.init_problem()
    y = prob.y_centres()
    k = 2 * math.pi / prob.meta["L"]
    basis = np.sin(k * y)

    def amp():
        ux = g.macro()["ux"][:, 0]
        return float(ux @ basis / (basis @ basis))

    a0 = amp()
    g.run(prob.nsteps)
    rate = -math.log(amp() / a0) / g.t
    nu_corr = analytic.viscosity(1.0, s6, dt)
    nu_plain = analytic.viscosity(1.0, s6)
    assert abs(rate / (nu_corr * k * k) - 1.0) < 0.01, (rate, nu_corr * k * k)
    assert abs(rate / (nu_plain * k * k) - 1.0) > 0.05


@pytest.mark.slow
@pytest.mark.parametrize("case,dx,ny,dt,E_paper", [(1, 0.004, 32, 1e-4, 0.0702), (2, 0.002, 64, 5e-5, 0.0386),
                                                   (3, 0.001, 128, 2.5e-5, 0.0206)])
def test_couette_reproduces_paper_errors(case, dx, ny, dt, E_paper):
    """Sect. V.D: plates at -+D/2 moving at -+U = 0.1, rho = T = 1, periodic
    in x; the paper reports E(u) = 7.02 %, 3.86 % and 2.06 % for its three
    cases (dx = 0.004, 0.002 and 0.001, s dt = 1, 0.5 and 0.25, t = 57.5).  Here the rates are
    divided and dt and t multiplied by ten, which keeps s dt, the lattice
    Courant number and nu t / D^2.  Walls sit on the ghost rows, so
    D = (ny + 1) dy.  Measured against the series with nu = T / s, the
    errors come out within 30 % of the printed ones and halve with dt like
    them."""
    s = 1e4
    prob = synth.couette(nx=4, ny=ny, dt=dt, U=0.1, noise=0.0, s_shear=s)
    prob.s = synth.rates(dt, default=s)
    prob.dx = prob.dy = dx
    prob.sides["south"] = synth.side("wall", (1.0, -0.1, 0.0, 1.0))
    prob.sides["north"] = synth.side("wall", (1.0, 0.1, 0.0, 1.0))
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(int(round(5.75 / dt)))
    u = g.macro()["ux"][:, 0]
    D = (ny + 1) * dx
    y = (np.arange(ny) + 1.0) * dx - D / 2
    E = metrics.paper_error(u, analytic.couette_paper(y, g.t, 0.1, D, analytic.viscosity(1.0, s)))
    assert abs(E / E_paper - 1.0) < 0.3, (E, E_paper)
    # the profile is antisymmetric about the centre line, as the set-up is
    np.testing.assert_allclose(u, -u[::-1], atol=1e-12)


def _shock_offsets(prob, mac, L, R, t):
    """Numerical minus exact position, in cells, of each shock of the exact
    solution (density midpoint crossing on the middle row)."""
    W = riemann.wave_speeds(L, R)
    x = prob.x_centres()
    J = prob.ny // 2
    out = {}
    for side, far in (("left", L[0]), ("right", R[0])):
        if W[side + "_shock"]:
            xs = prob.meta["x0"] + W[side + "_head"] * t
            level = 0.5 * (W["rho_star_" + side] + far)
            pos = metrics.crossing(x, mac["rho"][J], level, lo=xs - 0.1, hi=xs + 0.1)
            out[side] = None if pos is None else (pos - xs) / prob.dx
    return out


@pytest.mark.slow
def test_two_shock_collision_matches_exact_solution():
    """Sect. V.A(d), the paper's spacing, rates and time (t = 0.1): every
    relative error E below 1.5 % and both shocks within one cell."""
    prob = synth.two_shock()
    L, R = prob.meta["left"], prob.meta["right"]
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    E, mac, _ = _tube_errors(prob, g, L, R)
    assert max(E.values()) < 0.015, E
    off = _shock_offsets(prob, mac, L, R, g.t)
    assert set(off) == {"left", "right"} and all(abs(v) <= 1.0 for v in off.values()), off


@pytest.mark.slow
def test_two_shock_collision_mrt_oscillates_less_than_srt():
    """Sect. V.A(d): at the same spacing the MRT run (s5 = s6 = 5e3, s7 = s8 =
    3e4) oscillates less at the discontinuities than the single-relaxation-
    time run with tau = 1e-5.  Measured as the total variation in excess of
    the exact solution's, for rho, u, p and T: MRT's is below 0.6 of SRT's."""
    excess = {}
    for srt in (False, True):
        prob = synth.two_shock(srt=srt)
        g = core.Grid(prob, nthreads=8)
        g.init_problem()
        g.run(prob.nsteps)
        mac = g.macro()
        r, u, p, T = riemann.profile(prob.meta["left"], prob.meta["right"], prob.x_centres(),
                                     prob.meta["x0"], g.t, 2.0)
        J = prob.ny // 2
        excess[srt] = {k: np.sum(np.abs(np.diff(mac[k][J]))) - np.sum(np.abs(np.diff(ex)))
                       for k, ex in (("rho", r), ("ux", u), ("p", p), ("T", T))}
    for k in excess[False]:
        assert 0.0 < excess[False][k] < 0.6 * excess[True][k], (k, excess)


@pytest.mark.slow
def test_colella_explosion_matches_exact_solution():
    """Sect. V.A(c) at the paper's case-1 spacing (dx = 0.002, dt = 2e-6) and
    rates, run to t = 0.02 on an 800-cell tube (the full t = 0.1 run needs
    4000 cells and 50 000 steps: E = 0.96 / 0.25 / 0.20 / 0.46 % for rho, u,
    p, T there, against the paper's 1.69 / 1.60 / 1.11 / 0.78 %).  The
    T = 1000 | 0.01 jump: E below 4 % (rho), 3 % (u, p, T) and the shock
    within one cell."""
    prob = synth.colella(t_end=0.02, margins=(1.0, 0.6))
    L, R = prob.meta["left"], prob.meta["right"]
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    E, mac, _ = _tube_errors(prob, g, L, R)
    assert E["rho"] < 0.04 and E["ux"] < 0.03 and E["p"] < 0.03 and E["T"] < 0.03, E
    off = _shock_offsets(prob, mac, L, R, g.t)
    assert set(off) == {"right"} and abs(off["right"]) <= 1.0, off


def test_high_mach_tube_is_unstable_under_these_readings():
    """Sect. V.A(e) (Mach 10.1 | 6.3, dx = 0.003, dt = 1e-5, s5 = s6 = 1.5e4,
    s10 = 5e4): the paper reports a successful MRT run; with the readings
    taken here the west state (5, 45, 0, 10) has a growing mode (von Neumann
    screen: max |omega| = 1.019 per step in 1D), and the oracle goes to a
    negative temperature within 30 steps and to non-finite values before the
    run's 1800 steps end."""
    prob = synth.high_mach()
    g = core.Grid(prob, nthreads=4)
    g.init_problem()
    g.run(30)
    assert np.min(g.macro()["T"]) < 0.0
    g.run(prob.nsteps - 30)
    assert not np.all(np.isfinite(g.get_f()))


@pytest.mark.slow
def test_sod_reproduces_paper_errors():
    """Sect. V.A(a), case 1 (dx = 0.002, dt = 2e-6, t = 0.18): the paper
    prints E = 0.234 / 0.182 / 3.32 / 0.327 % for rho, p, u, T but not its
    tube length.  E of u counts only the disturbed region (u = 0 elsewhere),
    so it does not depend on the length: here 3.18 %.  The other three are
    divided by sums over the whole tube; fitting the undisturbed length on
    each side from E(rho) alone (the tube comes out ~7.8 long) predicts
    E(p) and E(T) within 3 % of the printed ones (0.180 % and 0.330 %)."""
    want = parse.paper_tube_errors()["sod_case1"]
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    prob = synth.sod(nx=int(round(1.0 / want["dx"])), dt=want["dt"], nsteps=int(round(0.18 / want["dt"])))
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    mac = g.macro()
    r, u, p, T = riemann.profile(L, R, prob.x_centres(), prob.meta["x0"], g.t, 2.0)
    J = prob.ny // 2
    ex = {"rho": r, "p": p, "ux": u, "T": T}
    far = {"rho": 1.0 + 0.125, "p": 1.0 + 0.1, "T": 1.0 + 0.8}
    num = {k: float(np.sum(np.abs(mac[k][J] - ex[k]))) for k in ex}
    den = {k: float(np.sum(np.abs(ex[k]))) for k in ex}
    assert abs(100 * num["ux"] / den["ux"] / want["ux"] - 1.0) < 0.1
    # extra undisturbed cells per side that give the printed E(rho)
    a = (100 * num["rho"] / want["rho"] - den["rho"]) / far["rho"]
    assert a > 0
    for k in ("p", "T"):
        e = 100 * num[k] / (den[k] + a * far[k])
        assert abs(e / want[k] - 1.0) < 0.03, (k, e, want[k])


@pytest.mark.slow
def test_lax_reproduces_paper_errors():
    """Sect. V.A(b), case 1 (dx = 0.004, dt = 4e-6, t = 0.2) on [0, 1.6]:
    all four E are divided by sums over the whole tube (u = 0.698 on the
    left), whose length the paper does not print.  Fitting the undisturbed
    length on each side from E(rho) alone gives a tube 7.5 long -- within
    5 % of the 7.8 the same fit gives for the Sod tube, so one tube length
    fits both printed tables -- and predicts E(p), E(u), E(T) within 20 %
    of the printed ones (0.191 / 0.505 / 0.325 % against 0.205 / 0.592 /
    0.310 %)."""
    want = parse.paper_tube_errors()["lax_case1"]
    prob = synth.lax(nx=400, length=1.6, dt=want["dt"], t_end=0.2)
    L, R = prob.meta["left"], prob.meta["right"]
    g = core.Grid(prob, nthreads=8)
    g.init_problem()
    g.run(prob.nsteps)
    mac = g.macro()
    r, u, p, T = riemann.profile(L, R, prob.x_centres(), prob.meta["x0"], g.t, 2.0)
    J = prob.ny // 2
    ex = {"rho": r, "p": p, "ux": u, "T": T}
    far = {"rho": L[0] + R[0], "p": L[2] + R[2], "ux": abs(L[1]) + abs(R[1]),
           "T": L[2] / L[0] + R[2] / R[0]}
    num = {k: float(np.sum(np.abs(mac[k][J] - ex[k]))) for k in ex}
    den = {k: float(np.sum(np.abs(ex[k]))) for k in ex}
    a = (100 * num["rho"] / want["rho"] - den["rho"]) / far["rho"]
    length = (prob.nx + 2 * a) * prob.dx
    assert abs(length / 7.8 - 1.0) < 0.05, length
    for k in ("p", "ux", "T"):
        e = 100 * num[k] / (den[k] + a * far[k])
        assert abs(e / want[k] - 1.0) < 0.2, (k, e, want[k])
