"""Von Neumann screen of a parameter set (Sect. IV), the FP64 numpy
reference of the library's mrtfd_screen.  TEST INFRASTRUCTURE ONLY (see
oracle/__init__.py).  The amplification matrix of one Fourier mode around
a uniform state,

  G = diag(1 - i a sin(th_x) + a^2 (cos th_x - 1) - i b sin(th_y) + b^2 (cos th_y - 1))
      - dt M^-1 S (M - d f-hat^eq / d f),

with a = v_x dt / dx, b = v_y dt / dy, and its largest eigenvalue modulus
over a grid of phases (k dx, k dy).  The scheme is linearly stable at that
state when max |omega| <= 1.  M and M^-1 are the oracle's (core.model); the
Jacobian of the equilibria (Eq. 14) is written out below; the eigenvalues
are numpy's.
"""
import numpy as np

from . import core


def model():
    m = core.model()
    return np.array(m.v, dtype=np.float64), np.array(m.M, dtype=np.float64), np.array(m.Minv, dtype=np.float64)


def feq_jacobian(rho, ux, uy, T):
    """d f-hat^eq_k / d (rho, j_x, j_y, e) at a state, from Eq. (14) with
    P = e - |j|^2 / (2 rho)."""
    jx, jy = rho * ux, rho * uy
    e = rho * (T + 0.5 * (ux * ux + uy * uy))
    r = 1.0 / rho
    J = np.zeros((16, 4))
    J[0, 0] = J[1, 1] = J[2, 2] = J[3, 3] = 1.0
    j2 = jx * jx + jy * jy
    P = e - 0.5 * j2 * r
    dP = np.array([0.5 * j2 * r * r, -jx * r, -jy * r, 1.0])  # dP/d(rho, jx, jy, e)
    # f5 = (jx^2 - jy^2)/rho
    J[4] = [-(jx * jx - jy * jy) * r * r, 2 * jx * r, -2 * jy * r, 0]
    # f6 = jx jy / rho
    J[5] = [-jx * jy * r * r, jy * r, jx * r, 0]
    # f7 = (e + P) jx / rho, f8 = (e + P) jy / rho
    h = e + P
    dh = dP + np.array([0, 0, 0, 1.0])
    J[6] = dh * jx * r + np.array([-h * jx * r * r, h * r, 0, 0])
    J[7] = dh * jy * r + np.array([-h * jy * r * r, 0, h * r, 0])
    # f9 = (jx^2 - 3 jy^2) jx / rho^2, f10 = (3 jx^2 - jy^2) jy / rho^2
    J[8] = [-2 * (jx ** 3 - 3 * jx * jy * jy) * r ** 3, (3 * jx * jx - 3 * jy * jy) * r * r, -6 * jx * jy * r * r, 0]
    J[9] = [-2 * (3 * jx * jx * jy - jy ** 3) * r ** 3, 6 * jx * jy * r * r, (3 * jx * jx - 3 * jy * jy) * r * r, 0]
    # f11 = 2 e^2 / rho - j2^2 / (4 rho^3)
    J[10] = [-2 * e * e * r * r + 0.75 * j2 * j2 * r ** 4, -j2 * jx * r ** 3, -j2 * jy * r ** 3, 4 * e * r]
    # f13 = (6 rho e - 2 j2)(jx^2 - jy^2) / rho^3, f14 = (6 rho e - 2 j2) jx jy / rho^3
    g = 6 * rho * e - 2 * j2
    dg = np.array([6 * e, -4 * jx, -4 * jy, 6 * rho])
    a13, a14 = jx * jx - jy * jy, jx * jy
    da13 = np.array([0, 2 * jx, -2 * jy, 0])
    da14 = np.array([0, jy, jx, 0])
    dr3 = np.array([-3 * r ** 4, 0, 0, 0])
    J[12] = dg * a13 * r ** 3 + g * da13 * r ** 3 + g * a13 * dr3
    J[13] = dg * a14 * r ** 3 + g * da14 * r ** 3 + g * a14 * dr3
    return J


def amplification(state, s, dx, dy, dt, theta_x, theta_y, mats=None):
    v, M, Minv = mats if mats is not None else model()
    Jf = feq_jacobian(*state) @ M[:4]
    coll = dt * Minv @ np.diag(np.asarray(s, dtype=np.float64)) @ (M - Jf)
    a = v[:, 0] * dt / dx
    b = v[:, 1] * dt / dy
    adv = (1 - 1j * a * np.sin(theta_x) + a * a * (np.cos(theta_x) - 1)
           - 1j * b * np.sin(theta_y) + b * b * (np.cos(theta_y) - 1))
    return np.diag(adv) - coll


def max_growth(state, s, dx, dy, dt, n=32):
    """(max |omega|, (theta_x, theta_y)) over a grid of phases in [0, pi] x
    [-pi, pi] (the other half follows by symmetry of real data)."""
    mats = model()
    best, where = -1.0, None
    for tx in np.linspace(0.0, np.pi, n + 1):
        for ty in np.linspace(-np.pi, np.pi, 2 * n + 1):
            w = np.max(np.abs(np.linalg.eigvals(amplification(state, s, dx, dy, dt, tx, ty, mats))))
            if w > best:
                best, where = float(w), (float(tx), float(ty))
    return best, where
