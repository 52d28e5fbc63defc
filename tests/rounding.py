"""FP32 rounding scales of the MRT step (test infrastructure): the
magnitudes that one FP32 step rounds against, from which the tests derive
their tolerances against the FP64 oracle.

* transform_scale: what the collision cancels down from;
* equilibrium_scale: the rounding of the conserved moments carried through
  the equilibria (Eq. 14) and the back-map;
* storage_field_bounds: what the storage rounding of the populations makes
  of rho, u1 and p after n steps (the tube-batch bounds).
"""
import numpy as np

from oracle import core


def transform_scale(prob, f):
    """max over nodes and populations of (|dt M^-1| |S| |M| |f|)_i + max_q |f_q|:
    the magnitude that the FP32 collision of a node cancels down from (the
    moments m_k = sum M_kq f_q and their equilibria, mapped back by dt M^-1 S),
    plus the node's own populations."""
    m = core.model()
    A = np.abs(m.Minv) * prob.dt @ np.diag(np.abs(prob.s)) @ np.abs(m.M)
    af = np.einsum("ik,kyx->iyx", A, np.abs(f))
    return float(np.max(af + np.max(np.abs(f), axis=0, keepdims=True)))


def equilibrium_scale(prob, f):
    """max over nodes of (|dt M^-1| |S| |d f-hat^eq / d c| |M_c| |f|)_i, c =
    (rho, j_x, j_y, e) and M_c their rows of M: the FP32 rounding of the
    conserved moments (a few u of |M_c| |f|) carried through the equilibria
    (Eq. 14) and the back-map.  Hot or fast states make it dominate
    transform_scale: populations of 1e4-1e5 sum to rho ~ 1-6 there.  The
    Jacobian is a central difference of the oracle's equilibria, once per
    distinct node state."""
    m = core.model()
    A = np.abs(m.Minv) * prob.dt @ np.diag(np.abs(prob.s))
    fl = f.reshape(16, -1)
    c = m.M[:4] @ fl
    cerr = np.abs(m.M[:4]) @ np.abs(fl)
    keys = np.round(np.concatenate([c, cerr]).T, 10)
    _, idx = np.unique(keys, axis=0, return_index=True)
    out = 0.0
    for i in idx:
        x0 = c[:, i]
        J = np.empty((16, 4))
        for k in range(4):
            h = 1e-6 * max(1.0, abs(x0[k]))
            xp, xm = x0.copy(), x0.copy()
            xp[k] += h
            xm[k] -= h
            J[:, k] = (core.feq_moments(*xp) - core.feq_moments(*xm)) / (2 * h)
        out = max(out, float(np.max(A @ np.abs(J) @ cerr[:, i])))
    return out


def storage_field_bounds(states, nsteps):
    """Per-node error bounds on (rho, u1, p) after nsteps FP32 steps of a flow
    made of the given macroscopic states (rho, u1, T), from the rounding of
    the stored populations.  Each step stores population i with an error of
    at most u/2 |f_i| (u = 2^-24; the step's increment is summed first, so
    this last rounding is the one at the scale of f); those of different
    steps are independent (round to nearest) and add as a random walk, sqrt(n)
    u/2 |f_i| after n steps.  The conserved moments sum them with weights
    (1, |v_i1|, |v_i|^2 / 2), and u1 = j1 / rho, p = e - j1^2 / (2 rho) (the
    model's gamma = 2) carry them on:
      d rho <= s sum_i |f_i|,  d j1 <= s sum_i |v_i1| |f_i|,
      d e <= s sum_i |v_i|^2/2 |f_i|,  s = sqrt(n) u / 2,
      d u1 <= (d j1 + |u1| d rho) / rho,  d p <= d e + |u1| d j1 + u1^2/2 d rho,
    with f = f^eq of each state; the maximum over the states is returned."""
    m = core.model()
    vx = np.abs(m.v[:, 0])
    v2 = 0.5 * np.sum(m.v ** 2, axis=1)
    s = np.sqrt(float(nsteps)) * 2.0 ** -24 / 2.0
    out = {"rho": 0.0, "ux": 0.0, "p": 0.0}
    for rho, u, T in states:
        f = np.abs(core.feq_velocity(rho, u, 0.0, T))
        drho, dj, de = s * f.sum(), s * (vx * f).sum(), s * (v2 * f).sum()
        out["rho"] = max(out["rho"], drho)
        out["ux"] = max(out["ux"], (dj + abs(u) * drho) / rho)
        out["p"] = max(out["p"], de + abs(u) * dj + 0.5 * u * u * drho)
    return out
