"""Evaluation of the learned P_5 closure on held-out random media.

For the held-out instances (closure seeds 2000 + i) the library runs the
high-order reference (default P_31), plain P_5, plain P_9 and P_5 with the
learned closure to t_final on the same grid, FP32 storage, and compares the
zeroth moment on G11 by relative L2 error against the reference.

Throughput: every model runs all instances as ONE batch (one graph launch,
the batch's autotuned tile; closure solvers use the batched fused closure
sweep), timed by device events around the graph launch (best of `repeats`
runs after an untimed one); the ratio of two models' times is their ratio of
throughput on the same work.  Single-instance times (graph-captured advance,
wall clock of the stepping loop) are reported beside it for a few instances,
for the closure model both with the network and the odd update as two kernels
(the single-solver default) and fused into one.

    python -m paper_1211_2205_amd.closure_eval --weights weights.npy --count 64
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def _make(prob, closure_params=None):
    import paper_1211_2205_amd as pa
    s = pa.Solver.from_problem(prob, precision="fp32", closure="learned" if closure_params is not None else "pn")
    if closure_params is not None:
        s.load_closure(closure_params)
    return s


def _batch(probs, closure_params=None, repeats=3):
    """All instances as one batch: zeroth moments at t_final, best device ms
    and wall ms of `repeats` timed runs, cell-moment updates of one run."""
    import paper_1211_2205_amd as pa
    solvers = [_make(p, closure_params) for p in probs]
    b = pa.Batch(solvers)
    b.autotune(2)
    b.run()  # untimed: capture
    best_ms = best_wall = math.inf
    rec = None
    for _ in range(repeats):
        b.reset()
        t0 = time.perf_counter()
        rec = b.run()
        best_wall = min(best_wall, (time.perf_counter() - t0) * 1e3)
        best_ms = min(best_ms, rec["ms"])
    r00 = [s.get_moment(0) for s in solvers]
    b.close()
    for s in solvers:
        s.close()
    return r00, best_ms, best_wall, rec["updates"]


def _single(prob, closure_params=None, fused=False):
    s = _make(prob, closure_params)
    if fused:
        s.set_closure_fused(True)
    s.run()  # untimed: device set-up and graph capture
    s.reset()
    s.synchronize()
    t0 = time.perf_counter()
    s.run()
    wall = time.perf_counter() - t0
    s.close()
    return wall


def _err(a, ref):
    return math.sqrt(float(np.sum((a - ref) ** 2)) / float(np.sum(ref ** 2)))


def evaluate(params, seeds, n=256, ref_order=31, singles=8, log=print):
    import workloads as wl
    seeds = list(seeds)
    runs = {}
    for label, N, cl in (("ref", ref_order, None), ("p5", 5, None), ("p9", 9, None), ("p5_closure", 5, params)):
        r00, ms, wall, upd = _batch([wl.closure_instance(k, N, n) for k in seeds], cl)
        runs[label] = {"r00": r00, "ms": ms, "wall_ms": wall, "updates": upd}
        log(f"closure eval: batch of {len(seeds)} {label}: {ms:.2f} ms device, {wall:.2f} ms wall")
    rows = []
    for i, k in enumerate(seeds):
        ref = runs["ref"]["r00"][i]
        row = {"seed_index": k, "err_p5": _err(runs["p5"]["r00"][i], ref), "err_p9": _err(runs["p9"]["r00"][i], ref),
               "err_p5_closure": _err(runs["p5_closure"]["r00"][i], ref)}
        rows.append(row)
        log(f"closure eval {k}: err P5 {row['err_p5']:.3e} P9 {row['err_p9']:.3e} "
            f"P5+closure {row['err_p5_closure']:.3e}")
    single = {}
    if singles > 0:
        for label, N, cl, fused in (("p5", 5, None, False), ("p9", 9, None, False), ("p5_closure", 5, params, False),
                                    ("p5_closure_fused", 5, params, True)):
            single[label] = float(np.mean([_single(wl.closure_instance(k, N, n), cl, fused)
                                           for k in seeds[:singles]]))
    e5 = np.array([r["err_p5"] for r in rows])
    e9 = np.array([r["err_p9"] for r in rows])
    ec = np.array([r["err_p5_closure"] for r in rows])
    summary = {
        "instances": len(rows), "n": n, "reference_order": ref_order,
        "mean_err_p5": float(e5.mean()), "mean_err_p9": float(e9.mean()), "mean_err_p5_closure": float(ec.mean()),
        "median_gain_vs_p5": float(np.median(e5 / ec)),
        "fraction_closure_better_than_p5": float(np.mean(ec < e5)),
        "fraction_closure_at_most_p9": float(np.mean(ec <= e9)),
        "batch_ms": {k: runs[k]["ms"] for k in runs}, "batch_wall_ms": {k: runs[k]["wall_ms"] for k in runs},
        "batch_updates": {k: runs[k]["updates"] for k in runs},
        "throughput_p5_closure_over_p9": runs["p9"]["ms"] / runs["p5_closure"]["ms"],
        "throughput_p5_over_p9": runs["p9"]["ms"] / runs["p5"]["ms"],
        "single_instances": min(singles, len(seeds)), "single_s": single,
        "single_throughput_p5_closure_over_p9": single["p9"] / single["p5_closure"] if single else None,
    }
    return summary, rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--weights", required=True)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--first", type=int, default=2000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--ref-order", type=int, default=31)
    ap.add_argument("--singles", type=int, default=8, help="instances timed one by one as well")
    ap.add_argument("--out", default=None, help="JSON with the summary and every instance")
    args = ap.parse_args(argv)
    params = np.load(args.weights, allow_pickle=False).astype(np.float32)
    summary, rows = evaluate(params, range(args.first, args.first + args.count), args.n, args.ref_order,
                             args.singles, log=lambda m: print(m, flush=True))
    print(json.dumps(summary), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "instances": rows}, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
