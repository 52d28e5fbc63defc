"""Exact solution of the 1D Riemann problem for an ideal gas (test infrastructure).

The paper compares its shock-tube runs with "exact solutions" (Sect. V.A)
without saying how they are obtained.  This is the textbook exact solver:
find the star pressure p* where the left and right wave curves meet, then
sample the self-similar solution at x/t.  Shocks follow the Rankine-Hugoniot
relations and rarefactions the isentropic fan.

The model's equation of state is that of a gas with two translational
degrees of freedom (e = rho (T + |u|^2/2), p = rho T), i.e. gamma = 2; gamma
is a parameter so that the solver can also be checked on gamma = 1.4 cases.
"""
import math

import numpy as np
from scipy.optimize import brentq


def sound_speed(rho, p, gamma):
    return math.sqrt(gamma * p / rho)


def _wave_curve(p, rhoK, pK, gamma):
    """f_K(p): velocity change across the K wave to reach pressure p."""
    aK = sound_speed(rhoK, pK, gamma)
    if p > pK:  # shock
        A = 2.0 / ((gamma + 1.0) * rhoK)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * aK / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def has_vacuum(left, right, gamma):
    rhoL, uL, pL = left
    rhoR, uR, pR = right
    aL, aR = sound_speed(rhoL, pL, gamma), sound_speed(rhoR, pR, gamma)
    return 2.0 / (gamma - 1.0) * (aL + aR) <= uR - uL


def star_state(left, right, gamma=2.0):
    """(p*, u*) of the Riemann problem with left/right = (rho, u, p)."""
    rhoL, uL, pL = left
    rhoR, uR, pR = right
    if has_vacuum(left, right, gamma):
        raise ValueError("Riemann problem generates vacuum")

    def g(p):
        return _wave_curve(p, rhoL, pL, gamma) + _wave_curve(p, rhoR, pR, gamma) + (uR - uL)

    lo, hi = 1e-14 * min(pL, pR), max(pL, pR)
    while g(hi) < 0.0:
        hi *= 2.0
    pstar = brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    ustar = 0.5 * (uL + uR) + 0.5 * (_wave_curve(pstar, rhoR, pR, gamma)
                                     - _wave_curve(pstar, rhoL, pL, gamma))
    return pstar, ustar


def _star_density(pstar, rhoK, pK, gamma):
    if pstar > pK:
        r = pstar / pK
        g = (gamma - 1.0) / (gamma + 1.0)
        return rhoK * (r + g) / (g * r + 1.0)
    return rhoK * (pstar / pK) ** (1.0 / gamma)


def wave_speeds(left, right, gamma=2.0):
    """Dict of the characteristic speeds: the left wave's head and tail, the
    contact, and the right wave's tail and head (equal for shocks)."""
    rhoL, uL, pL = left
    rhoR, uR, pR = right
    pstar, ustar = star_state(left, right, gamma)
    aL, aR = sound_speed(rhoL, pL, gamma), sound_speed(rhoR, pR, gamma)
    out = {"pstar": pstar, "ustar": ustar, "contact": ustar}
    if pstar > pL:
        S = uL - aL * math.sqrt((gamma + 1.0) / (2.0 * gamma) * pstar / pL + (gamma - 1.0) / (2.0 * gamma))
        out["left_head"] = out["left_tail"] = S
        out["left_shock"] = True
    else:
        out["left_head"] = uL - aL
        out["left_tail"] = ustar - aL * (pstar / pL) ** ((gamma - 1.0) / (2.0 * gamma))
        out["left_shock"] = False
    if pstar > pR:
        S = uR + aR * math.sqrt((gamma + 1.0) / (2.0 * gamma) * pstar / pR + (gamma - 1.0) / (2.0 * gamma))
        out["right_head"] = out["right_tail"] = S
        out["right_shock"] = True
    else:
        out["right_head"] = uR + aR
        out["right_tail"] = ustar + aR * (pstar / pR) ** ((gamma - 1.0) / (2.0 * gamma))
        out["right_shock"] = False
    out["rho_star_left"] = _star_density(pstar, rhoL, pL, gamma)
    out["rho_star_right"] = _star_density(pstar, rhoR, pR, gamma)
    return out


def sample(left, right, xi, gamma=2.0):
    """(rho, u, p) arrays of the exact solution at similarity variable xi = x/t."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rhoL, uL, pL = left
    rhoR, uR, pR = right
    W = wave_speeds(left, right, gamma)
    pstar, ustar = W["pstar"], W["ustar"]
    aL, aR = sound_speed(rhoL, pL, gamma), sound_speed(rhoR, pR, gamma)
    gm, gp = gamma - 1.0, gamma + 1.0
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s <= ustar:
            if s <= W["left_head"]:
                r, v, q = rhoL, uL, pL
            elif s >= W["left_tail"]:
                r, v, q = W["rho_star_left"], ustar, pstar
            else:  # inside the left fan
                v = 2.0 / gp * (aL + 0.5 * gm * uL + s)
                a = 2.0 / gp * (aL + 0.5 * gm * (uL - s))
                r = rhoL * (a / aL) ** (2.0 / gm)
                q = pL * (a / aL) ** (2.0 * gamma / gm)
        else:
            if s >= W["right_head"]:
                r, v, q = rhoR, uR, pR
            elif s <= W["right_tail"]:
                r, v, q = W["rho_star_right"], ustar, pstar
            else:  # inside the right fan
                v = 2.0 / gp * (-aR + 0.5 * gm * uR + s)
                a = 2.0 / gp * (aR - 0.5 * gm * (uR - s))
                r = rhoR * (a / aR) ** (2.0 / gm)
                q = pR * (a / aR) ** (2.0 * gamma / gm)
        rho[n], u[n], p[n] = r, v, q
    return rho, u, p


def profile(left, right, x, x0, t, gamma=2.0):
    """Exact (rho, u, p, T) at positions x for an interface at x0 and time t,
    with T = p / rho (R = 1)."""
    x = np.asarray(x, dtype=np.float64)
    if t <= 0.0:
        xi = np.where(x <= x0, -np.inf, np.inf)
    else:
        xi = (x - x0) / t
    rho, u, p = sample(left, right, xi, gamma)
    return rho, u, p, p / rho


def max_signal_speed(left, right, gamma=2.0):
    W = wave_speeds(left, right, gamma)
    return max(abs(W["left_head"]), abs(W["right_head"]), abs(W["left_tail"]), abs(W["right_tail"]))
