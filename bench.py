#!/usr/bin/env python3
"""Throughput of the staggered-grid P_N step on one MI355X.

Default workload: the large line source (P_39, 820 moments, 1000 x 1000
cells, FP64 storage as in the paper, CFL 0.5, t_final = 1: 666 steps), with
FP32 and BF16 storage as further legs.  A step is one full
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
SIZE = {"fp64": 8, "fp32": 4, "bf16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}


def _sweep_source_hash():
    with open(SWEEP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _pmc_record(precision, workload):
    """The committed HBM-counter summary of the sweep kernel for this workload
    and precision, if it was taken on the current kernel source; else None."""
    try:
        with open(PMC_SUMMARY.format(precision)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("sweep_source_sha256_16") != _sweep_source_hash() or rec.get("precision") != precision
            or rec.get("workload") != workload or "parity" not in rec):
        return None
    return rec


def _traffic(rec, variant, width, n_odd, n_even, alg_odd, alg_even):
    """HBM bytes per launch of this run, composed from the counter runs of each
    parity (one parity per counter run) with this run's own mix of odd and
    even launches; None unless the counters were taken on the same tile
    variant, m-range width and per-parity algorithmic bytes."""
    if rec is None or rec.get("variant") != variant or rec.get("width") != width:
        return None
    odd, even = rec["parity"].get("odd"), rec["parity"].get("even")
    if not odd or not even:
        return None
    for r, alg in ((odd, alg_odd), (even, alg_even)):
        if abs(r["algorithmic_bytes_per_launch"] - alg) > 1e-9 * alg:
            return None
    n = n_odd + n_even
    return (n_odd * odd["hbm_bytes_per_launch"] + n_even * even["hbm_bytes_per_launch"]) / n


def cpu_baseline(prob, rows, steps=1, rows_single=200):
    """Oracle (FP64, plain C + OpenMP) on a band of `rows` grid rows of the same
    workload (all of them: the workload itself) for `steps` full steps on all
    host threads, then one step on one thread on a band of `rows_single` rows
    (the oracle is memory-bound, a smaller band would sit in cache)."""
    import workloads as wl
    from oracle import scheme
    from oracle.scheme import OracleSolver
    h = (prob.ax[1] - prob.ax[0]) / prob.n[0]

    def run(r, k):
        if r >= prob.n[1]:
            band = wl.line_source(N=prob.N, n=prob.n[0], s=0.01, precision="fp64")
            what = f"the full {prob.n[0]} x {prob.n[1]} grid"
        else:
            band = wl.line_source(N=prob.N, n=prob.n[0], s=0.01, precision="fp64")
            band.n = (prob.n[0], r)
            band.ax = (prob.ax[0], prob.ax[1], -r * h / 2, r * h / 2)
            what = f"a {prob.n[0]} x {r} band"
        o = OracleSolver(band)
        o.evaluate_materials(0.0)
        t0 = time.perf_counter()
        for _ in range(k):
            o.step()
        t1 = time.perf_counter()
        updates = band.n[0] * band.n[1] * o.nmom * k
        del o
        return updates / (t1 - t0), (f"{k} full step(s) (4 half-steps each) of P_{prob.N} on {what} "
                                     f"({updates:.3e} cell-moment updates, {t1 - t0:.1f} s, FP64)")

    all_threads = scheme.set_threads(int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0)))
    v, sample = run(rows, steps)
    scheme.set_threads(1)
    v1, sample1 = run(rows_single, 1)
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
    achieved = rec["bytes"] / (rec["ms"] * 1e-3) / 1e9
    out = {"workload": f"random_media_batch_{count}_{precision}", "instances": count,
           "value": rec["updates"] / wall, "unit": "cell-moment updates/s",
           "device_ms": rec["ms"], "wall_ms": wall * 1e3, "launches": rec["launches"],
           "updates": rec["updates"], "groups": b.groups(),
           "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS}
    b.close()
    for x in solvers:
        x.close()
    return out


def closure_leg(count):
    """The learned closure (held-out random media 256^2, FP32): zeroth-moment
    error of plain P_5, plain P_9 and P_5 + closure against P_31, and the time
    of each model's batch of `count` instances (one graph launch)."""
    import numpy as np

    from paper_1211_2205_amd import closure_eval
    w = np.load(os.path.join(ROOT, "paper_1211_2205_amd", "weights", "closure_p5_256.npy"),
                allow_pickle=False).astype(np.float32)
    summary, _ = closure_eval.evaluate(w, range(2000, 2000 + count), singles=0, log=lambda m: None)
    summary["workload"] = f"closure_P5_256_heldout_{count}_fp32"
    return summary


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


def _tile_for(prec, workload, variant, width):
    """(variant, width) for the run: as given, else the pair the committed
    counter summary was taken on (the autotuner's choice when it was made, on
    the same kernel source), else None (autotune)."""
    if variant is not None:
        return variant, width
    rec = _pmc_record(prec, workload)
    if rec is not None:
        return rec["variant"], rec["width"]
    return None, width


def timed_run(prob, steps, warmup, variant=None, width=None):
    """One solver on prob: warmup untimed steps, then `steps` timed steps
    (wall clock around the advance call, and HIP events around every sweep
    launch on the solver's stream).  Returns the open solver and the record
    (value, roofline).  Keeps the solver at step warmup + steps."""
    import torch

    import paper_1211_2205_amd as pa
    prec = prob.precision
    workload = f"{prob.name}_{prec}"
    variant, width = _tile_for(prec, workload, variant, width)
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    if variant is None:
        s.autotune(2)
    else:
        if width:
            s.set_chunk_width(width)
        s.set_variant(variant)
    total = s.nsteps
    warm = max(0, min(warmup, total - 1))
    steps = total - warm if steps is None else min(steps, total - warm)
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
    # the same steps again from the initial state with the launches replayed
    # from HIP graphs (per-launch profiling is off): same end state, bit for bit
    s.reset()
    s.advance(warm)
    s.synchronize()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.advance(steps)
    s.synchronize()
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t2
    v, tx, ty = s.variant()
    w = s.chunk_width()
    # plain P_N, time-independent data: one advance of k steps launches the odd
    # sweep k + 1 times and the even sweep k times
    n_odd, n_even = steps + 1, steps
    b_odd, b_even = s.sweep_bytes(1), s.sweep_bytes(0)
    assert launches == n_odd + n_even and abs(n_odd * b_odd + n_even * b_even - alg_bytes) <= 1e-9 * alg_bytes
    updates = nx * ny * s.nmom * steps
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    per_launch = alg_bytes / launches
    avg_ms = kernel_ms / launches
    traffic = _traffic(_pmc_record(prec, workload), v, w, n_odd, n_even, b_odd, b_even)
    rec = {
        "value": updates / wall, "unit": "cell-moment updates/s", "steps": steps, "warmup": warm,
        "ms_per_step": wall / steps * 1e3, "dtype": DTYPE[prec],
        "config": {"workload": workload, "N": prob.N, "moments": s.nmom, "cells": [nx, ny],
                   "t_final": prob.t_final, "steps_to_t_final": total, "tile": [tx, ty], "variant": v,
                   "m_range_width": w, "sweeps_timed": launches, "odd_sweeps": n_odd, "even_sweeps": n_even},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "sweep_kernel", "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": per_launch,
                     "algorithmic_bytes_odd": b_odd, "algorithmic_bytes_even": b_even,
                     # HBM bytes of the counter runs over this run's launch time,
                     # the ratio of HBM to algorithmic bytes, and the design's
                     # 3 s bytes per cell-moment update at the measured rate
                     "hbm_GBs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                     "traffic_over_algorithmic": traffic / per_launch if traffic else None,
                     "effective_GBs": 3 * SIZE[prec] * updates / wall / 1e9},
        "graph_replay": {"value": updates / wall_graph, "ms_per_step": wall_graph / steps * 1e3},
    }
    return s, rec


def compare_states(a, b):
    """a against b (same problem, another storage precision), moment by
    moment through get_moment: relative L2 over all moments and points, the
    worst moment's relative L2 (its error over max(its norm, 1% of the largest
    moment norm)), and the largest pointwise error over max |b|."""
    num = den = 0.0
    errs, norms = [], []
    elem = scale = 0.0
    for k in range(b.nmom):
        gb = b.get_moment(k)
        d = a.get_moment(k) - gb
        e2, n2 = float((d * d).sum()), float((gb * gb).sum())
        num += e2
        den += n2
        errs.append(math.sqrt(e2))
        norms.append(math.sqrt(n2))
        elem = max(elem, float(abs(d).max()))
        scale = max(scale, float(abs(gb).max()))
    floor = 1e-2 * max(norms)
    per = [e / max(n, floor) for e, n in zip(errs, norms)]
    k = max(range(len(per)), key=per.__getitem__)
    return {"rel_l2": math.sqrt(num / den), "worst_moment": k, "worst_moment_rel_l2": per[k],
            "max_element_rel": elem / scale}


def ceiling_leg(gib):
    """Streaming ceilings of the device with plain library kernels (torch's
    own, on torch's current stream, timed with its events): a copy (1 read,
    1 write) and an elementwise add of two arrays into a third (2 reads, 1
    write: the sweep's mix of input, output-read and output-write bytes)."""
    import torch
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    out = {"bytes_per_array": 8 * n}
    for name, fn, nbytes in (("copy", lambda: c.copy_(a), 16 * n), ("add", lambda: torch.add(a, b, out=c), 24 * n)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def sweep_only(prob, parity, sweeps, variant, width):
    """Counter runs: `sweeps` single sweeps of one parity (tau = dt) on the
    workload's initial state, nothing else launched on the solver's stream
    after setup.  Prints the parity's algorithmic bytes per launch."""
    import torch

    import paper_1211_2205_amd as pa
    s = pa.Solver.from_problem(prob)
    s.bind_torch()
    if width:
        s.set_chunk_width(width)
    s.set_variant(variant)
    s.synchronize()
    torch.cuda.synchronize()
    p = 1 if parity == "odd" else 0
    s.sweep(p, s.dt, sweeps)
    s.synchronize()
    v, tx, ty = s.variant()
    print(json.dumps({"workload": f"{prob.name}_{prob.precision}", "parity": parity, "sweeps": sweeps,
                      "variant": v, "width": s.chunk_width(), "tile": [tx, ty],
                      "algorithmic_bytes_per_launch": s.sweep_bytes(p),
                      "sweep_source_sha256_16": _sweep_source_hash()}), flush=True)
    s.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the rest of the run)")
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--legs", default="fp32,bf16",
                    help="further storage precisions timed on the same workload, each with its own roofline "
                         "and its error against the headline's state at t_final (comma-separated; '' for none)")
    ap.add_argument("--variant", type=int, default=None,
                    help="sweep tile variant (default: the one of the committed counter summary, else autotune)")
    ap.add_argument("--width", type=int, default=None, help="m-range width with --variant")
    ap.add_argument("--cpu-rows", type=int, default=1000,
                    help="rows of the oracle's CPU sample (all rows: the whole workload)")
    ap.add_argument("--cpu-steps", type=int, default=6, help="full steps of the oracle's CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched leg (0: skip it)")
    ap.add_argument("--fused-steps", type=int, default=20,
                    help="timed steps of the parity-fused leg, P_7 on 1000^2 and 2048^2 (0: skip it)")
    ap.add_argument("--fused-orders", default="7", help="orders of the parity-fused leg (comma-separated)")
    ap.add_argument("--fused-cells", default="1000,2048", help="grid sizes n (n x n) of the parity-fused leg")
    ap.add_argument("--models-steps", type=int, default=20,
                    help="timed steps of the FP_N / D_N model leg (0: skip it)")
    ap.add_argument("--closure", type=int, default=16,
                    help="held-out instances of the learned-closure leg (0: skip it)")
    ap.add_argument("--ceiling-gib", type=float, default=2.0,
                    help="array size of the streaming-ceiling leg (torch copy and add; 0: skip it)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="only run a device copy of this size (HBM counter calibration) and exit")
    ap.add_argument("--sweep-only", choices=["odd", "even"], default=None,
                    help="only run --sweeps sweeps of one parity (HBM counter runs) and exit")
    ap.add_argument("--sweeps", type=int, default=8)
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

    import workloads as wl

    prob = wl.config(args.config, precision=args.precision)
    if args.sweep_only:
        variant, width = _tile_for(prob.precision, f"{prob.name}_{prob.precision}", args.variant, args.width)
        if variant is None:
            print("bench.py: --sweep-only needs --variant (and --width)", file=sys.stderr)
            sys.exit(2)
        sweep_only(prob, args.sweep_only, args.sweeps, variant, width)
        return

    s, head = timed_run(prob, args.steps, args.warmup, args.variant, args.width)
    diag = s.diagnostics()
    out = {
        "metric": "cell-moment updates/s",
        "value": head["value"],
        "unit": "cell-moment updates/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": head["warmup"],
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "graph_replay": head["graph_replay"],
        "state_check": {"mass": diag["mass"], "l2": diag["l2"], "nonfinite": diag["nonfinite"]},
    }
    legs = [p for p in args.legs.split(",") if p and p != prob.precision]
    if legs:
        # every leg runs on to t_final (untimed) and is compared with the
        # headline run's state there
        s.advance(s.nsteps - s.time()[2])
        s.synchronize()
        out["precisions"] = {}
        for prec in legs:
            lp = wl.config(args.config, precision=prec)
            ls, rec = timed_run(lp, args.steps, args.warmup, None if args.variant is None else args.variant,
                                args.width)
            ls.advance(ls.nsteps - ls.time()[2])
            ls.synchronize()
            rec["against_" + prob.precision + "_at_t_final"] = compare_states(ls, s)
            ls.close()
            out["precisions"][prec] = rec
    s.close()
    if args.ceiling_gib > 0:
        out["ceiling"] = ceiling_leg(args.ceiling_gib)
    if args.models_steps > 0:
        out["models"] = models_leg(args.config, prob.precision, args.models_steps)
    if args.fused_steps > 0:
        # 1000^2: one state copy (144 MB in FP32) stays in the 256 MB last-level
        # cache; 2048^2 (604 MB) does not
        out["fused"] = [fused_leg(int(N), int(n), prob.precision, args.fused_steps)
                        for N in args.fused_orders.split(",") for n in args.fused_cells.split(",")]
    if args.batch > 0:
        out["batch"] = batch_leg(args.batch, "fp32")
    if args.closure > 0:
        out["closure"] = closure_leg(args.closure)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_rows, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
