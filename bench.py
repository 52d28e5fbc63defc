#!/usr/bin/env python3
"""Throughput of the MRT finite-difference lattice Boltzmann step on one MI355X.

Default workload: the Mach-3 planar shock on a 30 degree wedge (the
Mach-reflection set-up of the paper's Sect. V.B(b)), 2048x512 nodes, FP32,
20000 steps.  A "step" is one pass of the whole hot path: boundary nodes,
then the fused collision + Lax-Wendroff + Euler update of every node.

Printed: one JSON line with MLUPS (node updates per second / 1e6), the
roofline of the step kernel (algorithmic 128 B per node update -- 16 FP32
populations read and written once -- over the kernel's own average launch
duration, against 8 TB/s HBM), the FP64 CPU oracle timed on a bounded crop of
the same workload, and the GPU crop run's error against that oracle.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % of HBM roofline (FP32 vs mixed vs batched) at stated L1 error"
HBM_PEAK_GBS = 8000.0
# VALU ceiling of the node update: the published FP32 vector rate, 157.3
# TFLOP/s = 256 CUs x 128 FP32 lanes x 2 (fused multiply-add) x 2.4 GHz,
# taken as 128 lane-operations per CU and clock (each add, multiply or fused
# multiply-add one operation), over about 330 operations per node update
# (factored transform)
ALU_NODE_RATE = 256 * 128 * 2.4e9 / 330
BYTES_PER_UPDATE = 128  # 16 FP32 populations read + 16 written
KERNEL_SRC = os.path.join(ROOT, "paper_0908_3749_amd", "csrc", "mrtfd_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def workloads():
    import synth

    return {
        # crop: the same set-up on a grid the oracle covers in 10-30 s for
        # cpu_steps steps (mach3: the geometry scaled by 1/4, wedge corner at
        # nx/4 as in the full grid)
        "mach3": dict(name="mach3_reflection_2048x512", make=lambda: synth.mach_reflection(),
                      crop=lambda: synth.mach_reflection(nx=512, ny=128), steps=20000, cpu_steps=10000),
        "bubble": dict(name="shock_bubble_4096x1024", make=lambda: synth.shock_bubble(),
                       crop=lambda: synth.shock_bubble(nx=512, ny=128), steps=10000, cpu_steps=10000),
        "couette": dict(name="couette_8192x2048", make=lambda: synth.couette(),
                        crop=lambda: synth.couette(x_window=(0, 16)), steps=50000, cpu_steps=20000),
        "sod": dict(name="sod_400x4", make=lambda: synth.sod(), crop=lambda: synth.sod(), steps=10000,
                    cpu_steps=10000),
        "tubes": dict(name="tube_batch_512", make=None, crop=None, steps=None),
    }


def tube_star(L, R):
    from oracle import riemann

    W = riemann.wave_speeds(L, R)
    return (riemann.max_signal_speed(L, R), min(W["rho_star_left"], W["rho_star_right"]),
            W["pstar"] / min(W["rho_star_left"], W["rho_star_right"]))


def bench_tubes(args):
    """512 seeded tubes in one batch (temporally blocked rounds), against the
    same tubes run one after another through the single-grid path (a sample,
    extrapolated by node updates), and the oracle on the smallest tubes."""
    import numpy as np
    import torch

    import synth
    from paper_0908_3749_amd import MRT2D, TubeBatch

    batch = synth.tube_batch(star_fn=tube_star)
    tubes = batch["tubes"]
    work = sum(4 * t["n"] * t["steps"] for t in tubes)
    B = TubeBatch.from_description(batch, use_graph=not args.no_graph)
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
    mlups = work / (ms * 1e-3) / 1e6
    # separate single-grid runs of a sample of tubes (graph-replayed steps)
    rng = np.random.default_rng(1)
    sample = sorted(rng.choice(len(tubes), size=8, replace=False).tolist())
    sep_ms, sep_work = 0.0, 0
    for k in sample:
        prob = synth.tube_problem(batch, k)
        n_steps = min(prob.nsteps, 4000)
        g = MRT2D.from_problem(prob, graph_steps=64)
        g.init_problem(prob)
        g.step(64)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(g.stream)
        g.step(n_steps)
        b.record(g.stream)
        torch.cuda.synchronize()
        sep_ms += a.elapsed_time(b)
        sep_work += 4 * prob.nx * n_steps
        g.close()
    sep_mlups = sep_work / (sep_ms * 1e-3) / 1e6
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": int(max(t["steps"] for t in tubes)), "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tube_batch_512", "ntubes": len(tubes), "rows": 4,
                   "node_updates": work, "seg_cols": seg, "round_steps": ks, "rounds": rounds,
                   "graph": not args.no_graph, "gamma": 2.0},
        "wall_ms": round(ms, 2), "setup_s": round(setup_s, 2),
        "roofline": {"bound": "alu", "achieved": round(work / (ms * 1e-3) / 1e9, 2),
                     "peak": round(ALU_NODE_RATE / 1e9, 1), "unit": "Gnode/s",
                     "frac": round(work / (ms * 1e-3) / ALU_NODE_RATE, 4), "traffic": None},
        "separate_launches": {"value": round(sep_mlups, 1), "unit": "MLUPS",
                              "sample": f"tubes {sample}, up to 4000 steps each, single-grid path, graph of 64 steps",
                              "speedup_batch": round(mlups / sep_mlups, 2)},
    }
    if not args.no_cpu:
        from oracle import core, metrics

        # the cheapest tubes, whole runs, until about 10 s of oracle time
        by_work = sorted(range(len(tubes)), key=lambda k: tubes[k]["n"] * tubes[k]["steps"])
        threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1, 16))
        cpu_s, cpu_work, acc, order = 0.0, 0, {}, []
        for k in by_work:
            if cpu_s >= 10.0 or len(order) >= 64:
                break
            order.append(k)
            prob = synth.tube_problem(batch, k)
            o = core.Grid(prob, nthreads=threads)
            o.init_problem()
            t0 = time.perf_counter()
            o.run(prob.nsteps)
            cpu_s += time.perf_counter() - t0
            cpu_work += 4 * prob.nx * prob.nsteps
            want = o.macro()
            got = B.macro_numpy(k)
            acc[f"tube{k}"] = {q: float(f"{metrics.rel_l1(got[q], want[q]):.3e}") for q in ("rho", "ux", "p")}
        out["cpu_baseline"] = {"value": round(cpu_work / cpu_s / 1e6, 3), "unit": "MLUPS", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{len(order)} tubes with the least work, whole runs, FP64, "
                                         f"{cpu_work:.3g} node updates in {cpu_s:.1f} s"}
        worst = {q: float(np.max([a[q] for a in acc.values()])) for q in ("rho", "ux", "p")}
        out["accuracy"] = {"against": "FP64 oracle, same tubes", "rel_l1_max_over_tubes": worst,
                           "non_finite_tubes": int(sum(not np.isfinite(a["rho"]) for a in acc.values())),
                           "rel_l1_first": dict(list(acc.items())[:4])}
    B.close()
    print(json.dumps(out), flush=True)
    return 0


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_entry(workload, kernel, seg, streaming, tile_order, per_launch_cells):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source, this workload and kernel variant."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    for e in rec.get("entries", []):
        if (e.get("source_sha") == kernel_sha() and e.get("workload") == workload
                and e.get("kernel") == kernel and int(e.get("rows", 0)) == int(seg)
                and bool(e.get("streaming", False)) == bool(streaming)
                and int(e.get("tile_order", 0)) == int(tile_order)):
            fetch = e["fetch_kib_per_dispatch"] * 1024 * e["copy_factor_fetch"]
            write = e["write_kib_per_dispatch"] * 1024 * e["copy_factor_write"]
            return {"bytes_per_launch": fetch + write,
                    "bytes_per_update": (fetch + write) / per_launch_cells}
    return None


def comparison():
    """The metric's three forms side by side in one run: Couette 8192x2048
    in plain FP32 and with the split-BF16x3 matrix-core transforms (1000
    timed steps each after 512 warm-up steps that hold the autotune and the
    graph capture), and the 512-tube batch (one whole run after a warm-up
    run).  Their accuracy against the oracle: bench.py --config couette
    [--precision bf16x3] and --config tubes."""
    import torch

    import synth
    from paper_0908_3749_amd import MRT2D, TubeBatch

    out = {}
    prob = synth.couette()
    cells = prob.nx * prob.ny
    for prec in ("fp32", "bf16x3"):
        g = MRT2D.from_problem(prob, graph_steps=64, precision=prec)
        g.init_problem(prob)
        g.step(512)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        n = 1000
        e0.record(g.stream)
        g.step(n)
        e1.record(g.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        kernel, seg, streaming, order = g.kernel_variant()
        g.close()
        gbs = BYTES_PER_UPDATE * cells / (ms * 1e-3) / 1e9
        out[prec] = {"workload": "couette_8192x2048", "value": round(cells / (ms * 1e-3) / 1e6, 1),
                     "unit": "MLUPS", "ms_per_step": round(ms, 6),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "kernel": f"{kernel}/{seg}{'/nt' if streaming else ''}{'/colbands' if order else ''}"}
    batch = synth.tube_batch(star_fn=tube_star)
    work = sum(4 * t["n"] * t["steps"] for t in batch["tubes"])
    B = TubeBatch.from_description(batch, use_graph=True)
    B.init()
    B.run()  # autotune, capture
    B.init()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(B.stream)
    B.run()
    e1.record(B.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out["batched"] = {"workload": "tube_batch_512", "value": round(work / (ms * 1e-3) / 1e6, 1),
                      "unit": "MLUPS", "wall_ms": round(ms, 2),
                      "alu_frac": round(work / (ms * 1e-3) / ALU_NODE_RATE, 4)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's run length)")
    ap.add_argument("--warmup", type=int, default=512,
                    help="untimed steps; they hold the kernel autotune (two passes over up to 9 "
                         "candidates, 360 steps at 2048x512) and the graph capture")
    ap.add_argument("--config", default="mach3", choices=sorted(workloads()))
    ap.add_argument("--kernel", default="auto", choices=["auto", "simple", "rows"])
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--graph-steps", type=int, default=64)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--layout", default="rows", choices=["rows", "planes", "tiles"])
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps on the crop (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle leg and the FP32 / mixed / batched comparison (profiling runs)")
    ap.add_argument("--flux-budget", type=int, default=1, choices=[0, 1],
                    help="1: after the headline run, time the same workload with the FP64 "
                         "outflow budget on (up to 2000 steps) and report it beside")
    ap.add_argument("--no-graph", action="store_true", help="tubes: launch rounds directly")
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

    from paper_0908_3749_amd import MRT2D

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
    if args.config == "tubes":
        return bench_tubes(args)
    W = workloads()[args.config]
    prob = W["make"]()
    steps = args.steps if args.steps is not None else W["steps"]
    cells = prob.nx * prob.ny

    def timed_run(flux_budget, nsteps):
        """Warm-up, then nsteps timed with HIP events on the context's stream.
        Returns (context, ms total, outflow-budget summary or None)."""
        g = MRT2D.from_problem(prob, kernel=args.kernel, rows=args.rows, graph_steps=args.graph_steps,
                               precision=args.precision, layout=args.layout, flux_budget=flux_budget)
        g.init_problem(prob)
        sums0 = g.sums()
        g.step(args.warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.step(nsteps)
        e1.record(g.stream)
        torch.cuda.synchronize()
        budget = None
        if flux_budget:
            sums = g.sums()
            out = g.outflow()
            resid = sums - sums0 + out.sum(axis=0)
            scale = abs(sums0) + abs(sums) + abs(out).sum(axis=0)
            kern, rows, nt, order = g.kernel_variant()
            budget = {"kernel": kern, "rows": rows, "streaming_stores": nt, "tile_order": order,
                      "outflow_total": [float(v) for v in out.sum(axis=0)],
                      "residual_over_scale": [float(f"{v:.3e}") for v in resid / scale]}
        return g, e0.elapsed_time(e1), budget

    g, ms_total, _ = timed_run(False, steps)
    ms_step = ms_total / steps
    mlups = cells * steps / (ms_total * 1e-3) / 1e6
    sums = g.sums()
    kernel, seg, streaming, tile_order = g.kernel_variant()
    g.close()
    budget = None
    if args.flux_budget:
        nb_steps = min(steps, 2000)
        gb, ms_b, summary = timed_run(True, nb_steps)
        gb.close()
        budget = {"value": round(cells * nb_steps / (ms_b * 1e-3) / 1e6, 1), "unit": "MLUPS",
                  "ms_per_step": round(ms_b / nb_steps, 6), "steps": nb_steps, **summary,
                  "note": "same workload with the FP64 outflow budget on (in leading blocks of "
                          "the step kernel's grid at one row per wave, else its own kernel on a "
                          "second stream beside each step); residual = sums(end) - sums(start) + outflow, "
                          "over warm-up and timed steps"}
    # One step = one launch of the step kernel (plus one single-thread clock
    # kernel per captured graph), so the kernel's average launch duration over
    # the timed region is the step time.
    k_ms = ms_step
    achieved = BYTES_PER_UPDATE * cells / (k_ms * 1e-3) / 1e9
    traffic = traffic_entry(W["name"], kernel, seg, streaming, tile_order, cells)
    print(f"bench: {W['name']} {steps} steps, {ms_step * 1e3:.2f} us/step, step kernel {kernel}"
          f"/{seg}{'/nt' if streaming else ''}{'/colbands' if tile_order else ''}, {mlups:.0f} MLUPS, "
          f"{achieved:.0f} GB/s",
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
        "dtype": "f32" if args.precision == "fp32" else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": W["name"], "nx": prob.nx, "ny": prob.ny, "dt": prob.dt,
                   "precision": args.precision, "layout": args.layout,
                   "kernel": kernel, "rows": seg, "streaming_stores": streaming,
                   "tile_order": tile_order,
                   "graph_steps": args.graph_steps,
                   "gamma": 2.0},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic["bytes_per_launch"]),
                     "kernel_us": round(k_ms * 1e3, 3),
                     "algorithmic_bytes_per_launch": BYTES_PER_UPDATE * cells},
        "fp64_sums": [float(v) for v in sums],
        "with_outflow_budget": budget,
    }

    if not args.no_cpu:
        from oracle import core, metrics

        crop = W["crop"]()
        n_cpu = args.cpu_steps if args.cpu_steps is not None else W["cpu_steps"]
        gc = MRT2D.from_problem(crop, kernel=args.kernel, rows=args.rows, precision=args.precision)
        gc.init_problem(crop)
        gc.step(n_cpu)
        got = gc.macro_numpy()
        gc.close()
        threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1, 16))
        o = core.Grid(crop, nthreads=threads)
        o.init_problem()
        t0 = time.perf_counter()
        o.run(n_cpu)
        cpu_s = time.perf_counter() - t0
        want = o.macro()
        out["cpu_baseline"] = {
            "value": round(crop.nx * crop.ny * n_cpu / cpu_s / 1e6, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"{crop.nx}x{crop.ny} crop of {W['name']} (same dx, dt, rates, boundary rules), "
                      f"{n_cpu} steps, FP64, {cpu_s:.1f} s",
        }
        out["accuracy"] = {
            "against": "FP64 oracle, same crop and steps",
            "rel_l1": {k: float(f"{metrics.rel_l1(got[k], want[k]):.3e}") for k in ("rho", "ux", "uy", "p")},
            "linf": {k: float(f"{metrics.linf(got[k], want[k]):.3e}") for k in ("rho", "ux", "uy", "p")},
        }
        if not np.all(np.isfinite(got["rho"])):
            out["accuracy"]["note"] = "non-finite values in the GPU crop run"
        if args.config == "mach3" and args.precision == "fp32":
            out["comparison"] = comparison()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
