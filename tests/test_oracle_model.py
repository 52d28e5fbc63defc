"""Pins of the oracle's model pieces against what the paper and mathematics fix:
the printed rows of M, M M^-1 = I, the equilibria as Maxwellian moments,
conservation by the collision, the equilibrium fixed point and the rate that
acts on each moment."""
import numpy as np
import pytest

from oracle import core
from tests.golden import parse

RNG = np.random.default_rng(20240908)


def moment_polys(vx, vy):
    """m_1..m_16 of Eq. (5a)-(5p) at arbitrary velocities (used only to take
    moments of a continuous Maxwellian; checked against the printed rows
    below)."""
    q = vx * vx + vy * vy
    x2, y2 = vx * vx, vy * vy
    return np.array([
        np.ones_like(vx), vx, vy, q / 2, x2 - y2, vx * vy, vx * q / 2, vy * q / 2,
        vx * (x2 - 3 * y2), vy * (3 * x2 - y2), q * q / 4, x2 * x2 - 6 * x2 * y2 + y2 * y2,
        q * (x2 - y2), q * vx * vy, vx * (x2 - 3 * y2) * q, vy * (3 * x2 - y2) * q])


def test_M_matches_printed_rows():
    m = core.model()
    printed = np.array(parse.printed_M())
    assert printed.shape == (16, 16)
    assert np.max(np.abs(m.M - printed)) <= 1e-13 * np.max(np.abs(printed))


def test_test_polynomials_match_printed_rows():
    m = core.model()
    printed = np.array(parse.printed_M())
    polys = moment_polys(m.v[:, 0], m.v[:, 1])
    assert np.max(np.abs(polys - printed)) <= 1e-12


def test_velocity_set_groups():
    v = core.model().v
    radii = np.hypot(v[:, 0], v[:, 1])
    np.testing.assert_allclose(radii, [1] * 4 + [6] * 4 + [2] * 4 + [3] * 4, rtol=0, atol=1e-15)
    # each group is closed under a quarter turn (vx, vy) -> (-vy, vx)
    for g in range(4):
        grp = v[4 * g:4 * g + 4]
        rot = np.stack([-grp[:, 1], grp[:, 0]], axis=1)
        for r in rot:
            assert np.min(np.hypot(*(grp - r).T)) < 1e-14


def test_inverse_is_inverse():
    m = core.model()
    assert np.max(np.abs(m.M @ m.Minv - np.eye(16))) <= 1e-13
    assert np.max(np.abs(m.Minv @ m.M - np.eye(16))) <= 1e-13
    # an independent inverse (LAPACK) agrees
    ref = np.linalg.inv(m.M)
    assert np.max(np.abs(m.Minv - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_oracle_inversion_on_known_matrix():
    A = np.array([[4.0, 3.0], [6.0, 3.0]])
    np.testing.assert_allclose(core.invert(A), [[-0.5, 0.5], [1.0, -2.0 / 3.0]], atol=1e-15)
    with pytest.raises(np.linalg.LinAlgError):
        core.invert(np.array([[1.0, 2.0], [2.0, 4.0]]))


def maxwellian_moments(rho, ux, uy, T, n=10):
    x, w = np.polynomial.hermite_e.hermegauss(n)  # weight exp(-x^2/2)
    X, Y = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w) / (2 * np.pi)
    VX, VY = ux + np.sqrt(T) * X, uy + np.sqrt(T) * Y
    return rho * np.tensordot(moment_polys(VX, VY), W, axes=([1, 2], [0, 1]))


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (0.125, 0.3, -0.7, 0.8),
                                   (2.3, 1.7, 0.4, 4.75), (0.445, 0.698, 0.0, 7.928)])
def test_equilibria_are_maxwellian_moments(state):
    """Eq. (14a)-(14i) are the moments of the 2D Maxwellian with R = 1 and
    e = rho (T + |u|^2/2); the paper sets moments 12, 15, 16 to zero."""
    rho, ux, uy, T = state
    e = rho * (T + 0.5 * (ux * ux + uy * uy))
    feq = core.feq_moments(rho, rho * ux, rho * uy, e)
    ref = maxwellian_moments(rho, ux, uy, T)
    keep = [k for k in range(16) if k not in (11, 14, 15)]
    np.testing.assert_allclose(feq[keep], ref[keep], rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
    assert feq[11] == 0.0 and feq[14] == 0.0 and feq[15] == 0.0


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (0.3, 0.4, -1.1, 2.5)])
def test_macro_roundtrip(state):
    rho, ux, uy, T = state
    q = core.macro_of(core.feq_velocity(rho, ux, uy, T))
    np.testing.assert_allclose(q, [rho, ux, uy, T, rho * T], rtol=1e-13, atol=1e-14)


def random_f():
    base = np.array([0.2] * 4 + [0.002] * 4 + [0.05] * 4 + [0.02] * 4)
    return base * (1 + 0.5 * RNG.uniform(-1, 1, 16))


def random_s():
    return np.concatenate([np.zeros(4), 10 ** RNG.uniform(2, 5, 12)])


def test_collision_conserves_mass_momentum_energy():
    m = core.model()
    for _ in range(50):
        f, s = random_f(), random_s()
        C = core.collision(f, s)
        mc = m.M @ C
        scale = np.abs(m.M) @ np.abs(C)
        assert np.all(np.abs(mc[:4]) <= 1e-12 * scale[:4] + 1e-300)
        assert np.max(np.abs(C)) > 1e-3  # the test data is far from equilibrium


def test_equilibrium_is_fixed_point():
    for state in [(1.0, 0.2, -0.1, 1.0), (3.0, 2.0, 1.0, 0.5), (0.2, -1.0, 0.0, 9.0)]:
        f = core.feq_velocity(*state)
        s = random_s()
        C = core.collision(f, s)
        assert np.max(np.abs(C)) <= 1e-13 * np.max(s) * np.max(np.abs(f))


@pytest.mark.parametrize("k", range(4, 16))
def test_rate_k_acts_on_moment_k(k):
    """Adding eps M^-1 e_k (k >= 5) to an equilibrium leaves rho, j, e
    unchanged, so the collision is exactly s_k eps M^-1 e_k."""
    m = core.model()
    f0 = core.feq_velocity(1.1, 0.3, -0.2, 0.9)
    eps = 1e-3
    f = f0 + eps * m.Minv[:, k]
    s = np.concatenate([np.zeros(4), np.arange(5, 17) * 1000.0])
    C = core.collision(f, s)
    expect = s[k] * eps * m.Minv[:, k]
    assert np.max(np.abs(C - expect)) <= 1e-9 * np.max(np.abs(expect))


def test_single_relaxation_time_reduction():
    """All rates equal: C = s (f - M^-1 f-hat^eq(f)) (Sect. II, S = I/tau)."""
    m = core.model()
    for _ in range(10):
        f = random_f()
        s0 = 3.7e4
        s = np.full(16, s0)
        C = core.collision(f, s)
        q = core.macro_of(f)
        feq = core.feq_velocity(q[0], q[1], q[2], q[3])
        np.testing.assert_allclose(C, s0 * (f - feq), rtol=1e-10, atol=1e-10 * s0 * np.max(np.abs(f)))
        assert m.M.shape == (16, 16)
