"""Readers for the text fixtures in this folder (no arithmetic of the method)."""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _token(tok):
    tok = tok.strip()
    parts = []
    cur = ""
    for ch in tok:
        if ch in "*/" and cur:
            parts.append(cur)
            cur = ch
        else:
            cur += ch
    parts.append(cur)
    val = float(int(parts[0]))
    for p in parts[1:]:
        op, arg = p[0], p[1:]
        x = math.sqrt(2.0) if arg == "r2" else float(int(arg))
        val = val * x if op == "*" else val / x
    return val


def printed_M():
    rows = []
    with open(os.path.join(HERE, "M_printed.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([_token(t) for t in line.split(",")])
    return rows


def paper_states():
    out = {}
    with open(os.path.join(HERE, "paper_states.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lab, *vals = line.split(",")
            out[lab] = [float(v) for v in vals]
    return out


def paper_tube_errors():
    """{label: dict(dx, dt, rho, p, ux, T)} with E in percent."""
    out = {}
    with open(os.path.join(HERE, "paper_tube_errors.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lab, dx, dt, r, p, u, T = line.split(",")
            out[lab] = dict(dx=float(dx), dt=float(dt), rho=float(r), p=float(p), ux=float(u), T=float(T))
    return out
