"""Closed-form references used to pin the oracle (test infrastructure).

* Couette flow (Sect. V.D): the paper's series for walls at +-D/2 moving at
  +-U, and the same construction for a resting bottom wall and a top wall
  moving at U.
* Transport coefficients: mu = rho R T / s (Eq. 15, 16) and their
  discretisation-corrected values mu' = rho R T (1/s + dt/2) (appendix).
* The amplification factor of the per-axis Lax-Wendroff difference with
  forward-Euler time marching for one Fourier mode (the advective part of the
  von Neumann matrix G, Sect. IV).
"""
import math

import numpy as np


def couette_paper(y, t, U, D, nu, nterms=2000):
    """Walls at y = -D/2 and +D/2 moving at -U and +U, fluid at rest at t = 0,
    kinematic viscosity nu = mu / rho (Sect. V.D)."""
    y = np.asarray(y, dtype=np.float64)
    u = 2.0 * y * U / D
    for j in range(1, nterms + 1):
        decay = math.exp(-4.0 * j * j * math.pi ** 2 * nu * t / (D * D))
        if decay == 0.0:
            break
        u = u - (-1.0) ** (j + 1) * 2.0 * U / (j * math.pi) * decay * np.sin(2.0 * j * math.pi * y / D)
    return u


def couette_one_wall(y, t, U, D, nu, nterms=2000):
    """Bottom wall at y = 0 at rest, top wall at y = D moving at U, fluid at
    rest at t = 0: the same sine-series construction on (0, D)."""
    y = np.asarray(y, dtype=np.float64)
    u = U * y / D
    for n in range(1, nterms + 1):
        decay = math.exp(-(n * math.pi) ** 2 * nu * t / (D * D))
        if decay == 0.0:
            break
        u = u - (-1.0) ** (n + 1) * 2.0 * U / (n * math.pi) * decay * np.sin(n * math.pi * y / D)
    return u


def viscosity(T, s, dt=0.0, R=1.0):
    """Kinematic viscosity mu/rho = R T (1/s + dt/2); dt = 0 gives the
    Chapman-Enskog value R T / s."""
    return R * T * (1.0 / s + 0.5 * dt)


def lw_amplification(c_x, c_y, theta_x, theta_y):
    """Growth factor per step of one Fourier mode exp(i(k_x x + k_y y)) under
    f <- f - dt v.grad f with the per-axis Lax-Wendroff difference, for
    Courant numbers c = v dt / dx and phases theta = k dx."""
    return (1.0 - 1j * c_x * math.sin(theta_x) + c_x * c_x * (math.cos(theta_x) - 1.0)
            - 1j * c_y * math.sin(theta_y) + c_y * c_y * (math.cos(theta_y) - 1.0))
