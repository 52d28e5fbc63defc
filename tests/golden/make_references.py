"""Writes the stored FP64 oracle references that the GPU tests and bench.py
compare against when the oracle itself would take too long on the test host.

Calls only the oracle (``oracle/``) and the seeded input generators
(``synth/``); nothing here touches the GPU library.

* ``couette``: the Couette flow of Sect. V.D as a 256 x 2048 window of the
  8192 x 2048 workload (the same per-cell velocity noise, periodic in x over
  the window), 50 000 steps (t = 0.5).  Stored: rho, u1, u2, p of the final
  state (FP32 roundings of the FP64 fields) and the oracle's wall time.
* ``mach15``: the Mach-1.5 reflection of Sect. V.B(b) at the paper's size
  (600 x 300, dx = 0.003, dt = 1e-5), 25 000 steps.  Stored: rho, u1, u2, p
  after 10 000 and 25 000 steps (FP32 roundings of the FP64 fields).
* ``tubes``: 16 tubes of the seeded 512-tube batch (seed 12345), each at
  its full CFL-limited run length: the shortest tube, the widest, the one
  that runs the most steps, the one that runs the fewest, and 12 drawn at
  random (seed 2026).  Stored per tube: rho, u1, p along one row (FP64; the
  tubes are y-uniform and the oracle's four rows are checked to be equal).

Usage: python tests/golden/make_references.py couette|mach15|tubes [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import core, riemann  # noqa: E402,F401

COUETTE_FILE = os.path.join(HERE, "couette_256x2048_50000.npz")
TUBES_FILE = os.path.join(HERE, "tube_sample_16.npz")
MACH15_FILE = os.path.join(HERE, "mach15_600x300.npz")
MACH15_STEPS = (10000, 25000)
COUETTE_WINDOW = (0, 256)
COUETTE_STEPS = 50000


def star_fn(L, R):
    W = riemann.wave_speeds(L, R)
    rmin = min(W["rho_star_left"], W["rho_star_right"])
    return riemann.max_signal_speed(L, R), rmin, W["pstar"] / rmin


def tube_sample(batch):
    """Indices of the sampled tubes, in the order described above."""
    tubes = batch["tubes"]
    n = np.array([t["n"] for t in tubes])
    st = np.array([t["steps"] for t in tubes])
    fixed = [int(np.argmin(n)), int(np.argmax(n)), int(np.argmax(st)), int(np.argmin(st))]
    rng = np.random.default_rng(2026)
    rest = [k for k in rng.permutation(len(tubes)).tolist() if k not in fixed][:12]
    return fixed + rest


def make_couette(threads):
    prob = synth.couette(x_window=COUETTE_WINDOW)
    o = core.Grid(prob, nthreads=threads)
    o.init_problem()
    t0 = time.perf_counter()
    done = 0
    while done < COUETTE_STEPS:
        n = min(5000, COUETTE_STEPS - done)
        o.run(n)
        done += n
        print(f"couette: {done} steps, {time.perf_counter() - t0:.0f} s", flush=True)
    wall = time.perf_counter() - t0
    m = o.macro()
    np.savez_compressed(COUETTE_FILE, steps=COUETTE_STEPS, window=np.array(COUETTE_WINDOW),
                        wall_s=wall, threads=threads,
                        **{k: m[k].astype(np.float32) for k in ("rho", "ux", "uy", "p")})
    print(f"wrote {COUETTE_FILE}", flush=True)


def make_mach15(threads):
    prob = synth.paper_mach_reflection()
    o = core.Grid(prob, nthreads=threads)
    o.init_problem()
    t0 = time.perf_counter()
    out = {}
    done = 0
    for stop in MACH15_STEPS:
        while done < stop:
            n = min(2500, stop - done)
            o.run(n)
            done += n
            print(f"mach15: {done} steps, {time.perf_counter() - t0:.0f} s", flush=True)
        m = o.macro()
        for k in ("rho", "ux", "uy", "p"):
            out[f"{k}_{stop}"] = m[k].astype(np.float32)
    np.savez_compressed(MACH15_FILE, steps=np.array(MACH15_STEPS), wall_s=time.perf_counter() - t0,
                        threads=threads, **out)
    print(f"wrote {MACH15_FILE}", flush=True)


def make_tubes(threads):
    batch = synth.tube_batch(star_fn=star_fn)
    sample = tube_sample(batch)
    out = {"index": np.array(sample), "n": [], "steps": [], "wall_s": []}
    fields = {"rho": [], "ux": [], "p": []}
    for k in sample:
        prob = synth.tube_problem(batch, k)
        o = core.Grid(prob, nthreads=threads)
        o.init_problem()
        t0 = time.perf_counter()
        o.run(prob.nsteps)
        wall = time.perf_counter() - t0
        m = o.macro()
        for q in fields:
            rows = m[q]
            assert np.array_equal(rows, np.broadcast_to(rows[0], rows.shape)), (k, q)
            fields[q].append(rows[0].copy())
        out["n"].append(prob.nx)
        out["steps"].append(prob.nsteps)
        out["wall_s"].append(wall)
        print(f"tube {k}: n {prob.nx}, steps {prob.nsteps}, {wall:.0f} s", flush=True)
    nmax = max(out["n"])
    packed = {}
    for q, rows in fields.items():
        a = np.full((len(sample), nmax), np.nan)
        for i, r in enumerate(rows):
            a[i, :len(r)] = r
        packed[q] = a
    np.savez_compressed(TUBES_FILE, index=out["index"], n=np.array(out["n"]),
                        steps=np.array(out["steps"]), wall_s=np.array(out["wall_s"]),
                        threads=threads, **packed)
    print(f"wrote {TUBES_FILE}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["couette", "mach15", "tubes"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    {"couette": make_couette, "mach15": make_mach15, "tubes": make_tubes}[a.what](a.threads)


if __name__ == "__main__":
    main()
