"""Error measures (test infrastructure).

* ``paper_error``: the relative error E = sum_I |num - exact| / sum_I |exact|
  along x at one row (Sect. V.A).
* ``rel_l1`` / ``linf``: element-wise comparison of two fields.
* ``crossing``: where a profile crosses a level, linearly interpolated
  between cell centres (used to locate shocks).
"""
import numpy as np


def paper_error(num, exact):
    num = np.asarray(num, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    return float(np.sum(np.abs(num - exact)) / np.sum(np.abs(exact)))


def rel_l1(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sum(np.abs(ref))
    return float(np.sum(np.abs(a - ref)) / den) if den > 0 else float(np.sum(np.abs(a - ref)))


def linf(a, ref):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(ref, dtype=np.float64))))


def crossing(x, y, level, lo=None, hi=None, last=True):
    """Position where y crosses level within x in [lo, hi]; the last crossing
    (largest x) when last is True, else the first.  None if none."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sel = np.ones_like(x, dtype=bool)
    if lo is not None:
        sel &= x >= lo
    if hi is not None:
        sel &= x <= hi
    idx = np.nonzero(sel)[0]
    found = []
    for a, b in zip(idx[:-1], idx[1:]):
        ya, yb = y[a] - level, y[b] - level
        if ya == 0.0:
            found.append(x[a])
        elif ya * yb < 0.0:
            found.append(x[a] + (x[b] - x[a]) * ya / (ya - yb))
    if not found:
        return None
    return found[-1] if last else found[0]
