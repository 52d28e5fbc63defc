"""FP32 rounding scales of the MRT step (test infrastructure): the
magnitudes that one FP32 step rounds against, from which the tests derive
their tolerances against the FP64 oracle.

* transform_scale: what the collision cancels down from;
* equilibrium_scale: the rounding of the conserved moments carried through
  the equilibria (Eq. 14) and the back-map;
* conserved_rounding: per node and step, the rounding of the conserved
  moments themselves, and what it makes of rho, u1 and p.
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
