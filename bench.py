#!/usr/bin/env python3
"""Throughput of the MRT finite-difference lattice Boltzmann step on one MI355X.

Default workload: Couette flow (the paper's Sect. V.D set-up with a resting
and a moving wall) on 8192 x 2048 nodes, FP32, stored as deviations from the
equilibrium at rest of rho = 1, T = 1 (2 x 1 GiB of populations: HBM-resident).
A "step" is one pass of the whole hot path: boundary nodes, then the fused
collision + Lax-Wendroff + Euler update of every node.

Timed region: K steps replayed from captured HIP graphs, after an untimed
set-up that lets the library's autotuner pick the step kernel (whatever
--warmup is) and W warm-up steps.

Printed: one JSON line with MLUPS (node updates per second / 1e6), the
roofline of the step kernel (algorithmic 128 B per node update -- 16 FP32
populations read and written once -- over the time per step, against 8 TB/s
HBM), the FP64 CPU oracle timed on a bounded sample of the same workload, the
accuracy of the FP32 and split-BF16x3 forms against the FP64 oracle at the
workload's full 50 000 steps (on a 256-column window of the grid, against a
stored oracle run), and the metric's other forms (Mach-3 reflection,
shock-bubble, split-BF16x3 Couette, the 512-tube batch) in `comparison`.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM roofline (FP32 vs mixed vs batched) at stated L1 error"
HBM_PEAK_GBS = 8000.0
# VALU ceiling of the node update.  The published FP32 vector rate, 157.3
# TFLOP/s = 256 CUs x 128 lanes x 2 x 2.4 GHz, counts packed FP32 (two lanes
# of work per instruction); the library is built without packed FP32, so a CU
# issues 64 FP32 lane-operations per clock (each add, multiply or fused
# multiply-add one operation): 256 x 64 x 2.4 GHz over about 330 operations
# per node update (factored transform) = 119 G node updates per second.
ALU_LANE_OPS_PER_CU_CLOCK = 64
OPS_PER_UPDATE = 330
ALU_NODE_RATE = 256 * ALU_LANE_OPS_PER_CU_CLOCK * 2.4e9 / OPS_PER_UPDATE
BYTES_PER_UPDATE = 128  # 16 FP32 populations read + 16 written
SETUP_STEPS = 1024      # untimed: covers the autotuner's trials (<= ~620 steps) and graph capture
KERNEL_SRCS = [os.path.join(ROOT, "paper_0908_3749_amd", "csrc", f) for f in ("mrtfd_kernels.hip", "mrtfd_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
COUETTE_REF = os.path.join(ROOT, "tests", "golden", "couette_256x2048_50000.npz")
TUBE_REF = os.path.join(ROOT, "tests", "golden", "tube_sample_16.npz")


def workloads():
    import synth

    return {
        # crop: the same set-up on a grid the oracle covers in 10-30 s for
        # cpu_steps steps (mach3: the geometry scaled by 1/4, wedge corner at
        # nx/4 as in the full grid); ref: the reference state at rest whose
        # equilibrium the library subtracts from the stored populations
        "couette": dict(name="couette_8192x2048", make=lambda: synth.couette(),
                        crop=lambda: synth.couette(x_window=(0, 256)), steps=50000, cpu_steps=None,
                        ref=(1.0, 1.0)),
        "mach3": dict(name="mach3_reflection_2048x512", make=lambda: synth.mach_reflection(),
                      crop=lambda: synth.mach_reflection(nx=512, ny=128), steps=20000, cpu_steps=10000,
                      ref=None),
        "bubble": dict(name="shock_bubble_4096x1024", make=lambda: synth.shock_bubble(),
                       crop=lambda: synth.shock_bubble(nx=512, ny=128), steps=10000, cpu_steps=10000,
                       ref=None),
        "sod": dict(name="sod_400x4", make=lambda: synth.sod(), crop=lambda: synth.sod(), steps=10000,
                    cpu_steps=10000, ref=None),
        "tubes": dict(name="tube_batch_512", make=None, crop=None, steps=None, ref=None),
    }


def host_threads():
    """(threads for the all-core oracle run, logical CPUs, CPUs this process
    may run on).  OMP_NUM_THREADS, where the host sets it, is this job's
    share of the machine."""
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = nproc
    env = os.environ.get("OMP_NUM_THREADS")
    threads = min(int(env), avail) if env and env.isdigit() and int(env) > 0 else avail
    return max(1, threads), nproc, avail


def kernel_sha():
    """sha256[:16] of the step kernels' code -- the kernel source and its
    internal header with comments and whitespace removed -- the key under
    which profiles/traffic.json holds the HBM counters."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_entry(workload, kernel, seg, streaming, tile_order, per_launch_cells, ref, precision="fp32"):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel code, this workload, precision and kernel
    variant."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    for e in rec.get("entries", []):
        if (e.get("source_sha") == kernel_sha() and e.get("workload") == workload
                and e.get("precision", "fp32") == precision
                and e.get("kernel") == kernel and int(e.get("rows", 0)) == int(seg)
                and bool(e.get("streaming", False)) == bool(streaming)
                and int(e.get("tile_order", 0)) == int(tile_order)
                and bool(e.get("reference", False)) == bool(ref)):
            fetch = e["fetch_kib_per_dispatch"] * 1024 * e["copy_factor_fetch"]
            write = e["write_kib_per_dispatch"] * 1024 * e["copy_factor_write"]
            return {"bytes_per_launch": fetch + write,
                    "bytes_per_update": (fetch + write) / per_launch_cells}
    return None


def timed_steps(prob, nsteps, warmup, graph_steps=64, ref=None, **kw):
    """Set-up (autotune, graph capture), warm-up, then nsteps timed with HIP
    events on the context's stream.  Returns (context, ms total, graph
    length used, FP64 sums of the initial state)."""
    import torch

    from paper_0908_3749_amd import MRT2D

    # the timed steps replay whole graphs: a graph no longer than the run
    G = min(int(graph_steps), nsteps - nsteps % 2) if graph_steps else 0
    g = MRT2D.from_problem(prob, graph_steps=max(G, 0), ref=ref, **kw)
    g.init_problem(prob)
    s0 = g.sums()
    g.step(SETUP_STEPS)
    if warmup:
        g.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step(nsteps)
    e1.record(g.stream)
    torch.cuda.synchronize()
    return g, e0.elapsed_time(e1), G, s0


def variant_name(v):
    kernel, seg, streaming, order = v
    return f"{kernel}/{seg}{'/nt' if streaming else ''}{'/colbands' if order else ''}"


def couette_accuracy():
    """The mixed-precision Couette workload at its stated length: a
    256-column window of the 8192 x 2048 Couette flow (same per-cell noise, periodic over the window; columns
    64..191 run on the matrix cores in the split-BF16x3 mode, nodes next to
    the walls and the window's first and last 64 columns on the FP32 path)
    for 50 000 steps in three forms, against the stored FP64 oracle run of
    the same window (tests/golden/make_references.py); and the x-averaged
    velocity profile against the one-moving-wall series of Sect. V.D."""
    import numpy as np

    import synth
    from oracle import analytic, metrics
    from paper_0908_3749_amd import MRT2D

    ref = np.load(COUETTE_REF)
    n = int(ref["steps"])
    crop = synth.couette(x_window=tuple(int(v) for v in ref["window"]))
    want = {k: ref[k].astype(np.float64) for k in ("rho", "ux", "uy", "p")}
    out = {"against": f"FP64 oracle, {crop.nx}x{crop.ny} window of couette_8192x2048, {n} steps "
                      f"(stored: {os.path.relpath(COUETTE_REF, ROOT)})", "steps": n}
    forms = {"fp32": dict(ref=(1.0, 1.0)), "bf16x3": dict(ref=(1.0, 1.0), precision="bf16x3"),
             "fp32_plain_storage": dict(ref=None)}
    got = {}
    for name, kw in forms.items():
        g = MRT2D.from_problem(crop, graph_steps=64, **kw)
        g.init_problem(crop)
        g.step(n)
        got[name] = g.macro_numpy()
        v = g.kernel_variant()
        g.close()
        m = got[name]
        out[name] = {"kernel": variant_name(v),
                     "rel_l1": {k: float(f"{metrics.rel_l1(m[k], want[k]):.3e}") for k in want},
                     "linf": {k: float(f"{metrics.linf(m[k], want[k]):.3e}") for k in want}}
    # the matrix-core window: interior tiles differ from the FP32 run, the
    # wall rows and edge tile columns (FP32 path in both) agree closely
    d = np.abs(got["bf16x3"]["ux"] - got["fp32"]["ux"])
    out["bf16x3"]["mfma_columns"] = [64, crop.nx - 64]
    out["bf16x3"]["max_abs_ux_diff_vs_fp32"] = {
        "mfma_tiles": float(f"{d[4:-4, 64:crop.nx - 64].max():.3e}"),
        "fp32_tiles": float(f"{np.concatenate([d[:, :64], d[:, crop.nx - 64:]], axis=1).max():.3e}")}
    # profile: x-average of u1 against the series with nu' = T (1/s + dt/2)
    U, D, t = crop.meta["U"], crop.meta["D"], n * crop.dt
    y = (np.arange(crop.ny) + 1.0) * crop.dy  # walls on the ghost rows, y = 0 and D
    nu = analytic.viscosity(1.0, crop.s[5], crop.dt)
    series = analytic.couette_one_wall(y, t, U, D, nu)
    prof = {"series_nu": nu, "t": t}
    for name, m in (("oracle", want), ("fp32", got["fp32"]), ("bf16x3", got["bf16x3"])):
        prof[f"E_u_{name}_vs_series"] = float(f"{metrics.paper_error(m['ux'].mean(axis=1), series):.4e}")
    prof["max_abs_profile_fp32_vs_oracle"] = float(
        f"{np.max(np.abs(got['fp32']['ux'].mean(axis=1) - want['ux'].mean(axis=1))):.3e}")
    out["profile"] = prof
    return out


def cpu_baseline(crop, seconds=8.0):
    """The FP64 oracle on crop: one thread, then all of this job's threads,
    each for about `seconds` of steps."""
    from oracle import core

    threads, nproc, avail = host_threads()
    res = {}
    for label, th in (("single_thread", 1), ("all_cores", threads)):
        o = core.Grid(crop, nthreads=th)
        o.init_problem()
        o.run(2)  # first touch of the arrays
        steps, t0 = 0, time.perf_counter()
        chunk = 5 if th == 1 else 50
        while time.perf_counter() - t0 < seconds:
            o.run(chunk)
            steps += chunk
        dt = time.perf_counter() - t0
        res[label] = (crop.nx * crop.ny * steps / dt / 1e6, steps, dt, th)
    v, steps, dt, th = res["all_cores"]
    v1, steps1, dt1, _ = res["single_thread"]
    return {"value": round(v, 3), "unit": "MLUPS", "cores": th, "kind": "oracle",
            "sample": f"{crop.nx}x{crop.ny} window of the workload (same dx, dt, rates, boundary rules), "
                      f"FP64: {steps} steps on {th} threads in {dt:.1f} s; {steps1} steps on 1 thread in "
                      f"{dt1:.1f} s",
            "single_thread": round(v1, 3), "host_nproc": nproc, "host_cpus_available": avail}


def bench_batch(with_separate=True, with_accuracy=True, no_graph=False):
    """The 512 seeded tubes in one batch (temporally blocked rounds; one
    whole run after a warm-up run that holds the autotune and the graph
    capture); against the same tubes run through the single-grid path (a
    stratified sample, whole runs, extrapolated by node updates); and the
    sampled tubes against their stored FP64 oracle runs."""
    import numpy as np
    import torch

    import synth
    from paper_0908_3749_amd import MRT2D, TubeBatch

    batch = synth.tube_batch(star_fn=synth.tube_star)
    tubes = batch["tubes"]
    work = sum(4 * t["n"] * t["steps"] for t in tubes)
    B = TubeBatch.from_description(batch, use_graph=not no_graph)
    t0 = time.perf_counter()
    B.init()
    B.run()  # autotune, capture; also the warm-up
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    B.init()
    torch.cuda.synchronize()
    e0.record(B.stream)
    B.run()
    e1.record(B.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    seg, ks, rounds = B.info()
    rate = work / (ms * 1e-3)
    out = {"workload": "tube_batch_512", "value": round(rate / 1e6, 1), "unit": "MLUPS",
           "wall_ms": round(ms, 2), "setup_s": round(setup_s, 2), "node_updates": work,
           "seg_cols": seg, "round_steps": ks, "rounds": rounds, "graph": not no_graph,
           "roofline": {"bound": "alu", "achieved": round(rate / 1e9, 2),
                        "peak": round(ALU_NODE_RATE / 1e9, 1), "unit": "Gnode/s",
                        "frac": round(rate / ALU_NODE_RATE, 4), "traffic": None}}
    if with_separate:
        # stratified by node updates: one tube from each eighth of the work
        # distribution, each run whole through the single-grid path
        order = sorted(range(len(tubes)), key=lambda k: tubes[k]["n"] * tubes[k]["steps"])
        sample = [order[(2 * i + 1) * len(order) // 16] for i in range(8)]
        sep_ms, sep_work = 0.0, 0
        for k in sample:
            prob = synth.tube_problem(batch, k)
            g = MRT2D.from_problem(prob, graph_steps=64)
            g.init_problem(prob)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(g.stream)
            g.step(prob.nsteps)
            b.record(g.stream)
            torch.cuda.synchronize()
            sep_ms += a.elapsed_time(b)
            sep_work += 4 * prob.nx * prob.nsteps
            g.close()
        sep = sep_work / (sep_ms * 1e-3) / 1e6
        out["separate_launches"] = {
            "value": round(sep, 1), "unit": "MLUPS", "speedup_batch": round(rate / 1e6 / sep, 2),
            "sample": f"tubes {sample} (one per eighth of the work distribution), whole runs, "
                      f"single-grid path, graph of 64 steps; {sep_work:.3g} node updates in {sep_ms:.0f} ms"}
    if with_accuracy and os.path.exists(TUBE_REF):
        from oracle import metrics

        ref = np.load(TUBE_REF)
        acc, shock, weak = {}, [], []
        for i, k in enumerate(ref["index"].tolist()):
            n = int(ref["n"][i])
            got = B.macro_numpy(k)
            want = {q: ref[q][i, :n] for q in ("rho", "ux", "p")}
            acc[k] = {q: metrics.rel_l1(got[q][0], want[q]) for q in want}
            prob = synth.tube_problem(batch, k)
            W = synth.riemann_waves(tubes[k]["left"], tubes[k]["right"])
            x = prob.x_centres()
            for side, far in (("left", tubes[k]["left"][0]), ("right", tubes[k]["right"][0])):
                if W[side + "_shock"]:
                    xs = prob.meta["x0"] + W[side + "_head"] * prob.t_end
                    lvl = 0.5 * (W["rho_star_" + side] + far)
                    a = metrics.crossing(x, want["rho"], lvl, lo=xs - 6 * prob.dx, hi=xs + 6 * prob.dx)
                    b = metrics.crossing(x, got["rho"][0], lvl, lo=xs - 6 * prob.dx, hi=xs + 6 * prob.dx)
                    if a is not None and b is not None:
                        # jumps below a tenth of the pre-shock density place
                        # their midpoint by the field error over the jump
                        strong = (W["rho_star_" + side] - far) / far >= 0.1
                        (shock if strong else weak).append(abs(a - b) / prob.dx)
        out["accuracy"] = {
            "against": f"FP64 oracle, {len(acc)} sampled tubes at full length "
                       f"(stored: {os.path.relpath(TUBE_REF, ROOT)})",
            "rel_l1_max_over_tubes": {q: float(f"{max(a[q] for a in acc.values()):.3e}") for q in ("rho", "ux", "p")},
            "rel_l1_median_over_tubes": {q: float(f"{np.median([a[q] for a in acc.values()]):.3e}")
                                         for q in ("rho", "ux", "p")},
            "shocks_jump_at_least_0.1": len(shock),
            "max_shock_offset_cells": float(f"{max(shock):.3e}") if shock else None,
            "weaker_shocks": len(weak),
            "max_weaker_shock_offset_cells": float(f"{max(weak):.3e}") if weak else None}
    B.close()
    return out


# FP64 flops per matrix of the von Neumann screen at the Fig. 2 state,
# counted on a replica of the kernel's steps: balancing and the Householder
# reduction ~5.0e4, ~42 shifted QR steps ~9.7e4.
SCREEN_FLOPS_PER_MATRIX = 1.5e5
FP64_VECTOR_PEAK_TFLOPS = 78.6


def bench_screen(reps=20, cpu_sample=200):
    """The von Neumann screen (Sect. IV) at the Fig. 2 state over a 65 x 129
    phase grid (8385 matrices): the kernel timed with HIP events on the
    stream it runs on, the numpy screen (the oracle's matrix, LAPACK's
    eigenvalues, one host core) timed on the first cpu_sample matrices, and
    the agreement of max |omega| between the two on that sample."""
    import numpy as np
    import torch

    import synth
    from paper_0908_3749_amd import stability

    state, dx, dt = (2.0, 10.0, 0.0, 2.0), 2e-3, 1e-5
    s = synth.rates(dt, s5=6500, s7=9e4, s8=9e4, s9=8e4, s13=7e4, s14=8e3, s15=2.5e4)
    th = stability.phase_grid(64)
    n = th.shape[0]
    d_th = torch.from_numpy(np.ascontiguousarray(th)).cuda()
    d_rho = torch.empty(n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    stability.screen_into(state, s, dx, dx, dt, d_th, d_rho, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        stability.screen_into(state, s, dx, dx, dt, d_th, d_rho, stream=stream)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rho = d_rho.cpu().numpy()
    from oracle import stability as ref  # the numpy screen, timed beside

    mats = ref.model()
    t0 = time.perf_counter()
    want = np.array([np.max(np.abs(np.linalg.eigvals(ref.amplification(state, s, dx, dx, dt, a, b, mats))))
                     for a, b in th[:cpu_sample]])
    cpu_s = time.perf_counter() - t0
    tflops = SCREEN_FLOPS_PER_MATRIX * n / (ms * 1e-3) / 1e12
    return {"value": round(n / (ms * 1e-3), 1), "unit": "matrices/s", "matrices": n, "ms_per_call": round(ms, 4),
            "max_omega": float(rho.max()),
            "roofline": {"bound": "alu", "achieved": round(tflops, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
                         "flops_per_matrix": SCREEN_FLOPS_PER_MATRIX,
                         "note": "bound by each matrix's chain of dependent rotations, not by the FP64 rate"},
            "cpu_baseline": {"value": round(cpu_sample / cpu_s, 1), "unit": "matrices/s", "cores": 1,
                             "kind": "oracle", "sample": f"the first {cpu_sample} of the same matrices, numpy"},
            "max_rel_diff_vs_numpy": float(f"{np.max(np.abs(rho[:cpu_sample] - want) / want):.3e}"),
            "config": "state (2, 10, 0, 2), dx = dy = 2e-3, dt = 1e-5, the printed MRT rates (Fig. 2), "
                      "phase pairs over [0, pi] x [-pi, pi]"}


def comparison(warmup):
    """The metric's other forms in the same run: the Mach-3 reflection
    (2048x512, cache-resident) and the shock-bubble (4096x1024) in FP32, the
    Couette 8192x2048 with the split-BF16x3 matrix-core transforms and in
    FP64 (populations stored in FP64: 256 B per node update), each 2000
    timed steps after the set-up and warm-up; the 512-tube batch; and the
    von Neumann screen of Sect. IV."""
    import synth

    out = {}
    cases = (("mach3_reflection_2048x512", synth.mach_reflection(), {}),
             ("shock_bubble_4096x1024", synth.shock_bubble(), {}),
             ("couette_8192x2048_bf16x3", synth.couette(), dict(ref=(1.0, 1.0), precision="bf16x3")),
             ("couette_8192x2048_fp64", synth.couette(), dict(ref=(1.0, 1.0), precision="fp64")))
    for name, prob, kw in cases:
        n = 2000
        g, ms, G, _ = timed_steps(prob, n, warmup, **kw)
        v = g.kernel_variant()
        g.close()
        cells = prob.nx * prob.ny
        step_ms = ms / n
        per_node = 2 * BYTES_PER_UPDATE if kw.get("precision") == "fp64" else BYTES_PER_UPDATE
        out[name] = {"value": round(cells * n / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
                     "ms_per_step": round(step_ms, 6),
                     "hbm_frac": round(per_node * cells / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "bytes_per_node_update": per_node,
                     "kernel": variant_name(v), "steps": n, "graph_steps": G}
    out["batched"] = bench_batch()
    out["stability_screen_fig2_8385"] = bench_screen()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's run length)")
    ap.add_argument("--warmup", type=int, default=512,
                    help="untimed warm-up steps, after an untimed set-up of 1024 steps that holds the "
                         "kernel autotune and the graph capture")
    ap.add_argument("--config", default="couette", choices=sorted(workloads()))
    ap.add_argument("--kernel", default="auto", choices=["auto", "simple", "rows"])
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=64)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp64"])
    ap.add_argument("--layout", default="rows", choices=["rows", "planes", "tiles"])
    ap.add_argument("--no-ref", action="store_true", help="store f itself (no reference state)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps on the crop for the accuracy of --config mach3/bubble/sod")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle legs, the accuracy runs and the comparison (profiling runs)")
    ap.add_argument("--flux-budget", type=int, default=1, choices=[0, 1],
                    help="1: after the headline run, time the same workload with the FP64 "
                         "outflow budget on (up to 2000 steps) and report it beside")
    ap.add_argument("--no-graph", action="store_true", help="tubes: launch rounds directly")
    ap.add_argument("--screen", action="store_true",
                    help="only time the von Neumann screen (as in the comparison) and print it")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only time a plain device copy of MIB MiB (the reference for the HBM "
                         "byte counters and for achievable bandwidth) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: the library runs on one GPU only (asked for {max(args.gpus, world)}); "
              "the multi-GPU slab decomposition is a design, not an implementation.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_mib": args.calibrate_copy, "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "ms": round(ms, 4), "gbs_read_plus_write": round(8 * n / ms / 1e6, 1)}), flush=True)
        return 0
    if args.screen:
        print(json.dumps(bench_screen()), flush=True)
        return 0
    if args.config == "tubes":
        out = bench_batch(with_separate=not args.no_cpu, with_accuracy=not args.no_cpu,
                          no_graph=args.no_graph)
        line = {"metric": METRIC, "value": out["value"], "unit": "MLUPS", "n_gpus": 1, "steps": None,
                "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "tube_batch_512", "ntubes": 512, "rows": 4,
                           "seg_cols": out["seg_cols"], "round_steps": out["round_steps"],
                           "rounds": out["rounds"], "graph": out["graph"], "gamma": 2.0},
                **{k: v for k, v in out.items() if k not in ("value", "unit", "workload")}}
        print(json.dumps(line), flush=True)
        return 0

    W = workloads()[args.config]
    prob = W["make"]()
    steps = args.steps if args.steps is not None else W["steps"]
    ref = None if args.no_ref else W["ref"]
    cells = prob.nx * prob.ny
    kw = dict(kernel=args.kernel, rows=args.rows, precision=args.precision, layout=args.layout)

    g, ms_total, G, _ = timed_steps(prob, steps, args.warmup, args.graph_steps, ref=ref, **kw)
    ms_step = ms_total / steps
    mlups = cells * steps / (ms_total * 1e-3) / 1e6
    sums = g.sums()
    kernel, seg, streaming, tile_order = g.kernel_variant()
    g.close()

    budget = None
    if args.flux_budget:
        nb_steps = min(steps, 2000)
        gb, ms_b, _, s0 = timed_steps(prob, nb_steps, 0, args.graph_steps, ref=ref, flux_budget=True, **kw)
        # sums and outflow over the set-up and timed steps
        s1 = gb.sums()
        out_b = gb.outflow()
        kb = gb.kernel_variant()
        gb.close()
        resid = s1 - s0 + out_b.sum(axis=0)
        scale = np.abs(s0) + np.abs(s1) + np.abs(out_b).sum(axis=0)
        budget = {"value": round(cells * nb_steps / (ms_b * 1e-3) / 1e6, 1), "unit": "MLUPS",
                  "ms_per_step": round(ms_b / nb_steps, 6), "steps": nb_steps, "kernel": variant_name(kb),
                  "outflow_total": [float(v) for v in out_b.sum(axis=0)],
                  "residual_over_scale": [float(f"{v:.3e}") for v in resid / scale],
                  "note": "same workload with the FP64 outflow budget on (in leading blocks of the step "
                          "kernel's grid at one row per wave, else its own kernel on a second stream "
                          "beside each step); residual = sums(end) - sums(start) + outflow over all steps"}

    per_node = 2 * BYTES_PER_UPDATE if args.precision == "fp64" else BYTES_PER_UPDATE
    achieved = per_node * cells / (ms_step * 1e-3) / 1e9
    traffic = traffic_entry(W["name"], kernel, seg, streaming, tile_order, cells, ref, args.precision)
    print(f"bench: {W['name']} {steps} steps, {ms_step * 1e3:.2f} us/step, step kernel "
          f"{variant_name((kernel, seg, streaming, tile_order))}, {mlups:.0f} MLUPS, {achieved:.0f} GB/s",
          file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3+f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": W["name"], "nx": prob.nx, "ny": prob.ny, "dt": prob.dt,
                   "precision": args.precision, "layout": args.layout,
                   "stored": "f - f^eq(rho=%g, u=0, T=%g)" % ref if ref else "f",
                   "kernel": kernel, "rows": seg, "streaming_stores": streaming,
                   "tile_order": tile_order, "graph_steps": G,
                   "setup_steps_untimed": SETUP_STEPS, "gamma": 2.0},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic["bytes_per_launch"]),
                     "step_us": round(ms_step * 1e3, 3),
                     "algorithmic_bytes_per_launch": per_node * cells,
                     "timing": "HIP events on the context's stream around the timed steps: one step-kernel "
                               "launch per step plus one single-thread clock kernel per replayed graph"},
        "fp64_sums": [float(v) for v in sums],
        "with_outflow_budget": budget,
    }

    if not args.no_cpu:
        if args.config == "couette" and args.precision == "fp32" and ref is not None:
            out["accuracy"] = couette_accuracy()
            out["cpu_baseline"] = cpu_baseline(W["crop"]())
            out["comparison"] = comparison(args.warmup)
        else:
            from oracle import core, metrics
            from paper_0908_3749_amd import MRT2D

            crop = W["crop"]()
            n_cpu = args.cpu_steps if args.cpu_steps is not None else (W["cpu_steps"] or 1000)
            gc = MRT2D.from_problem(crop, ref=ref, **kw)
            gc.init_problem(crop)
            gc.step(n_cpu)
            got = gc.macro_numpy()
            gc.close()
            threads, nproc, avail = host_threads()
            o = core.Grid(crop, nthreads=threads)
            o.init_problem()
            t0 = time.perf_counter()
            o.run(n_cpu)
            cpu_s = time.perf_counter() - t0
            want = o.macro()
            out["cpu_baseline"] = {
                "value": round(crop.nx * crop.ny * n_cpu / cpu_s / 1e6, 3), "unit": "MLUPS",
                "cores": threads, "kind": "oracle", "host_nproc": nproc, "host_cpus_available": avail,
                "sample": f"{crop.nx}x{crop.ny} crop of {W['name']} (same dx, dt, rates, boundary rules), "
                          f"{n_cpu} steps, FP64, {cpu_s:.1f} s"}
            out["accuracy"] = {
                "against": "FP64 oracle, same crop and steps",
                "rel_l1": {k: float(f"{metrics.rel_l1(got[k], want[k]):.3e}") for k in ("rho", "ux", "uy", "p")},
                "linf": {k: float(f"{metrics.linf(got[k], want[k]):.3e}") for k in ("rho", "ux", "uy", "p")}}
            if not np.all(np.isfinite(got["rho"])):
                out["accuracy"]["note"] = "non-finite values in the GPU crop run"
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
