#!/usr/bin/env python3
"""Throughput of the staggered-grid P_N step on one MI355X.

Default workload: the large line source (P_39, 820 moments, 1000 x 1000
cells, FP32 storage, CFL 0.5, t_final = 1: 666 steps).  A step is one full
time step of every moment (odd and even parity sweeps); the first `warmup`
steps of the run are untimed and the remaining `steps` are timed, so the
default covers exactly the run to t_final.

Prints one JSON line: cell-moment updates/s (nx * ny * moments * steps /
wall time of the timed steps), the sweep kernel's achieved algorithmic HBM
bandwidth against the 8 TB/s peak (HIP events around every launch, on the
stream the kernels run on), and the oracle's throughput on a bounded sample
of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "sweep_line_source_P39_1000_{}_pmc.json")
SWEEP_SRC = os.path.join(ROOT, "paper_1211_2205_amd", "csrc", "sweep.hip")


def _sweep_source_hash():
    with open(SWEEP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(launch_bytes, precision):
    """HBM bytes per launch from the committed PMC summary, if it was taken on
    the current sweep kernel source; else None."""
    try:
        with open(PMC_SUMMARY.format(precision)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256_16") != _sweep_source_hash() or rec.get("precision") != precision:
        return None
    if abs(rec.get("algorithmic_bytes_per_launch", 0.0) - launch_bytes) > 1e-6 * launch_bytes:
        return None  # counters taken on another workload
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(prob, rows):
    """Oracle (FP64, plain C + OpenMP) on a band of `rows` grid rows of the same
    workload for one full step, on all host threads, then on one thread (the
    same band: the oracle is memory-bound, a smaller band would sit in cache)."""
    import workloads as wl
    from oracle import scheme
    from oracle.scheme import OracleSolver
    h = (prob.ax[1] - prob.ax[0]) / prob.n[0]

    def run(r):
        band = wl.line_source(N=prob.N, n=prob.n[0], s=0.01, precision="fp64")
        band.n = (prob.n[0], r)
        band.ax = (prob.ax[0], prob.ax[1], -r * h / 2, r * h / 2)
        o = OracleSolver(band)
        o.evaluate_materials(0.0)
        t0 = time.perf_counter()
        o.step()
        t1 = time.perf_counter()
        updates = prob.n[0] * r * o.nmom
        return updates / (t1 - t0), (f"one full step (4 half-steps) of P_{prob.N} on a {prob.n[0]} x {r} band "
                                     f"({updates:.3e} cell-moment updates, {t1 - t0:.1f} s, FP64)")

    all_threads = scheme.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0)))
    v, sample = run(rows)
    scheme.set_threads(1)
    v1, sample1 = run(rows)
    scheme.set_threads(all_threads)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": v, "unit": "cell-moment updates/s", "cores": all_threads, "kind": "oracle",
            "cpu_model": model, "sample": sample,
            "single_thread": {"value": v1, "unit": "cell-moment updates/s", "cores": 1, "sample": sample1}}


def batch_leg(count, precision):
    """The heterogeneous batch (count random media, N in {3,5,7,9}, n in
    64..512, t_final 0.5): every instance run to t_final by one graph launch of
    the batched sweep; one untimed run first, then a timed one from t = 0."""
    import paper_1211_2205_amd as pa
    import workloads as wl
    probs = wl.batch(count, precision)
    solvers = [pa.Solver.from_problem(p) for p in probs]
    b = pa.Batch(solvers)
    b.autotune(2)
    b.run()
    b.reset()
    t0 = time.perf_counter()
    rec = b.run()
    wall = time.perf_counter() - t0
    v, w = b.variant()
    achieved = rec["bytes"] / (rec["ms"] * 1e-3) / 1e9
    out = {"workload": f"random_media_batch_{count}_{precision}", "instances": count,
           "value": rec["updates"] / wall, "unit": "cell-moment updates/s",
           "device_ms": rec["ms"], "wall_ms": wall * 1e3, "launches": rec["launches"],
           "updates": rec["updates"], "tile_variant": v, "m_range_width": w,
           "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS}
    b.close()
    for x in solvers:
        x.close()
    return out


def models_leg(config, precision, steps):
    """The moment models of the paper's outlook on the same workload: plain
    P_N, filtered P_N (damping 10 (l/(N+1))^4 per order: the decay planes
    change, the kernels do not), diffusion-corrected P_N (kappa = 0.1 dx:
    each step adds an even sweep split and the diffusion kernels on the N + 1
    order-N moments), and time-dependent absorption in separable form (per
    step the decay planes are combined on the device and the odd half-steps
    no longer merge).  Per model: updates/s over `steps` timed steps after
    two untimed ones, each solver autotuned."""
    import torch

    import paper_1211_2205_amd as pa
    import workloads as wl
    out = {}
    for model in ("pn", "fpn", "dn", "separable"):
        prob = wl.config(config, precision=precision)
        if model == "fpn":
            prob.filter_damping = wl.filter_damping(prob.N, 10.0)
        elif model == "dn":
            h = (prob.ax[1] - prob.ax[0]) / prob.n[0]
            prob.diffusion = (lambda k: (lambda t, x, y: k + 0 * x))(0.1 * h)
        elif model == "separable":
            # time-dependent absorption 0.1 (1 + 0.5 sin(2 pi t)) (1 + x^2) in separable form
            term = (lambda t: 0.1 * (1.0 + 0.5 * math.sin(2.0 * math.pi * t)), lambda x, y: 1.0 + x * x + 0 * y)
            prob.separable = {"absorption": [term]}
            prob.sigma_a = lambda t, x, y: term[0](t) * term[1](x, y)
            prob.time_dependent = True
        s = pa.Solver.from_problem(prob)
        s.bind_torch()
        s.autotune(1)
        s.advance(2)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps)
        s.synchronize()
        wall = time.perf_counter() - t0
        nx, ny = prob.n
        v, tx, ty = s.variant()
        out[model] = {"value": nx * ny * s.nmom * steps / wall, "unit": "cell-moment updates/s",
                      "ms_per_step": wall / steps * 1e3, "steps": steps, "tile": [tx, ty]}
        s.close()
    out["workload"] = f"{wl.config(config).name}_{precision}"
    return out


def fused_leg(N, n, precision, steps):
    """Parity-fused passes against the separate sweeps on a line source of
    order N on n x n cells: ms per step for both (autotuned separate sweeps),
    and the fused pass's algorithmic bandwidth, 2 s bytes per moment and point
    per step (each moment read and written once)."""
    import torch

    import paper_1211_2205_amd as pa
    import workloads as wl
    out = {"workload": f"line_source_P{N}_{n}_{precision}"}
    for mode in ("separate", "fused"):
        prob = wl.line_source(N=N, n=n, s=0.03, precision=precision)
        prob.t_final = 1.0
        s = pa.Solver.from_problem(prob)
        if mode == "fused":
            s.set_fused(True)
        s.bind_torch()
        if mode == "separate":
            s.autotune(1)
        s.advance(2)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps)
        s.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        rec = {"ms_per_step": ms, "value": n * n * s.nmom * steps / (ms * steps * 1e-3),
               "unit": "cell-moment updates/s"}
        if mode == "fused":
            pts = 0
            for k in range(s.nmom):
                nx, ny, _, _ = s.moment_shape(k)
                pts += nx * ny
            size = {"fp64": 8, "fp32": 4, "bf16": 2}[precision]
            gbs = 2 * size * pts / (ms * 1e-3) / 1e9
            rec.update({"algorithmic_bytes_per_step": 2 * size * pts, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS})
        out[mode] = rec
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the rest of the run)")
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--variant", type=int, default=None, help="sweep tile variant (default: autotune)")
    ap.add_argument("--cpu-rows", type=int, default=200, help="rows of the oracle's CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched leg (0: skip it)")
    ap.add_argument("--fused-steps", type=int, default=20,
                    help="timed steps of the parity-fused leg, P_7 on 1000^2 and 2048^2 (0: skip it)")
    ap.add_argument("--fused-orders", default="7", help="orders of the parity-fused leg (comma-separated)")
    ap.add_argument("--fused-cells", default="1000,2048", help="grid sizes n (n x n) of the parity-fused leg")
    ap.add_argument("--models-steps", type=int, default=20,
                    help="timed steps of the FP_N / D_N model leg (0: skip it)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="only run a device copy of this size (HBM counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the decomposition over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * 2 ** 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    import paper_1211_2205_amd as pa
    import workloads as wl

    prob = wl.config(args.config, precision=args.precision)
    prec = prob.precision
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    if args.variant is None:
        s.autotune(2)
    else:
        s.set_variant(args.variant)
    total = s.nsteps
    warm = max(0, min(args.warmup, total - 1))
    steps = args.steps if args.steps is not None else total - warm
    nmom = s.nmom
    nx, ny = prob.n

    s.advance(warm)
    s.synchronize()
    torch.cuda.synchronize()
    s.profile_begin()
    t0 = time.perf_counter()
    s.advance(steps)
    s.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms, launches, alg_bytes = s.profile_end()
    wall = t1 - t0
    diag = s.diagnostics()

    updates = nx * ny * nmom * steps
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    per_launch = alg_bytes / launches
    v, tx, ty = s.variant()
    traffic = _traffic(per_launch, prec)
    out = {
        "metric": "cell-moment updates/s",
        "value": updates / wall,
        "unit": "cell-moment updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{prob.name}_{prec}", "N": prob.N, "moments": nmom, "cells": [nx, ny],
                   "t_final": prob.t_final, "steps_to_t_final": total, "tile": [tx, ty],
                   "sweeps_timed": launches},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "sweep_kernel", "avg_launch_ms": kernel_ms / launches,
                     "algorithmic_bytes_per_launch": per_launch,
                     # HBM bytes of the counter runs over this run's launch time, and
                     # the design's 3 s bytes per cell-moment update at the measured rate
                     "hbm_GBs": traffic / (kernel_ms / launches * 1e-3) / 1e9 if traffic else None,
                     "effective_GBs": 3 * {"fp64": 8, "fp32": 4, "bf16": 2}[prec] * updates / wall / 1e9},
        "state_check": {"mass": diag["mass"], "l2": diag["l2"], "nonfinite": diag["nonfinite"]},
    }
    s.close()
    if args.models_steps > 0:
        out["models"] = models_leg(args.config, prec, args.models_steps)
    if args.fused_steps > 0:
        # 1000^2: one state copy (144 MB in FP32) stays in the 256 MB last-level
        # cache; 2048^2 (604 MB) does not
        out["fused"] = [fused_leg(int(N), int(n), prec, args.fused_steps)
                        for N in args.fused_orders.split(",") for n in args.fused_cells.split(",")]
    if args.batch > 0:
        out["batch"] = batch_leg(args.batch, "fp32")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
