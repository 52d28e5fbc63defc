"""Finds the draws of the seeded tube batch that the method cannot run and
prints them for synth.UNRUNNABLE_DRAWS.

Calls only the oracle and the input generators.  Each tube of the batch runs
in the FP64 oracle on a window of `window` columns around its initial jump
(same states, rates and spacing; the window's ends carry the end states as
the full tube's do, and no wave reaches them in the screened steps) for
min(steps, its own run length) steps; a tube fails if rho or T is
non-positive or non-finite anywhere at one of the checks (every `every`
steps).  Failed draws are skipped and the batch is drawn again until every
tube passes.

Usage: python tests/golden/screen_tubes.py [--window 600] [--steps 2000] [--procs 8]
"""
import argparse
import copy
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import core, riemann  # noqa: E402


def star_fn(L, R):
    W = riemann.wave_speeds(L, R)
    rmin = min(W["rho_star_left"], W["rho_star_right"])
    return riemann.max_signal_speed(L, R), rmin, W["pstar"] / rmin


def runs(args):
    batch, k, window, steps, every = args
    b = copy.deepcopy(batch)
    b["tubes"][k]["n"] = window
    prob = synth.tube_problem(b, k)
    o = core.Grid(prob, nthreads=1)
    o.init_problem()
    n = min(steps, batch["tubes"][k]["steps"])
    done = 0
    while done < n:
        m = min(every, n - done)
        o.run(m)
        done += m
        q = o.macro()
        if not (np.all(np.isfinite(q["rho"])) and np.all(np.isfinite(q["T"]))
                and q["rho"].min() > 0 and q["T"].min() > 0):
            return k, done
    return k, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--window", type=int, default=600)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--seed", type=int, default=12345)
    a = ap.parse_args()
    skip = set()
    screened = set()
    with Pool(a.procs) as pool:
        while True:
            batch = synth.tube_batch(seed=a.seed, star_fn=star_fn, skip_draws=tuple(sorted(skip)))
            todo = [k for k, t in enumerate(batch["tubes"]) if t["draw"] not in screened]
            bad = []
            for k, fail in pool.imap_unordered(runs, [(batch, k, a.window, a.steps, a.every) for k in todo]):
                screened.add(batch["tubes"][k]["draw"])
                if fail is not None:
                    t = batch["tubes"][k]
                    print(f"draw {t['draw']} (tube {k}): fails by step {fail}; L {np.round(t['left'], 3)} "
                          f"R {np.round(t['right'], 3)}", flush=True)
                    bad.append(t["draw"])
            if not bad:
                break
            skip.update(bad)
            print(f"{len(bad)} new failing draws; drawing again", flush=True)
    print(f"seed {a.seed}: UNRUNNABLE_DRAWS = {tuple(sorted(skip))}", flush=True)


if __name__ == "__main__":
    main()
