"""Training of the learned P_5 closure on the GPU.

Data: high-order (default P_31) runs of the random-media problems on an
n x n grid (default 256), t_final 0.5, FP32 storage, from the library's
solver.  At a number of snapshot times each run contributes closure inputs and
targets (the order-6 flux the truncation to P_5 drops, scaled by dx / nu) at
random cells, extracted by the library's sample kernel.

Training: the library's network trainer (BF16-MFMA forward and backward,
Adam), mean squared error, cosine learning-rate decay, a held-out fraction of
the samples for validation.  The closure is first fitted to snapshots of the
high-order solution (a-priori).  It acts, however, inside the P_5 scheme on
P_5 states, which drift from the truncated high-order states; so in rounds of
"closure in the loop" (--loop-rounds) the current network runs inside P_5 on
training instances next to the high-order run, and the P_5 + closure states
at the snapshot times become further inputs, paired with the high-order
run's order-6 flux at the same cells (rescaled to the P_5 stencil norm),
before the network is trained further on all samples.  At full strength the
closure can still amplify grid-scale modes (it is a centred, explicitly
integrated flux term of the order-5 moments themselves); the output layer is
therefore scaled by a factor alpha chosen a posteriori on training instances.
Writes the FP32 parameter blob (.npy) and a JSON log.

    python -m paper_1211_2205_amd.closure_train --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

N_IN, N_HIDDEN, N_OUT, N_FEATURES = 128, 128, 6, 101


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases; the
    padded inputs of the first layer get zero weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = np.zeros((N_HIDDEN, N_IN))
    W1[:, :N_FEATURES] = rng.uniform(-1, 1, size=(N_HIDDEN, N_FEATURES)) / math.sqrt(N_FEATURES)
    W2 = rng.uniform(-1, 1, size=(N_HIDDEN, N_HIDDEN)) / math.sqrt(N_HIDDEN)
    W3 = rng.uniform(-1, 1, size=(N_OUT, N_HIDDEN)) / math.sqrt(N_HIDDEN)
    parts = [W1, np.zeros(N_HIDDEN), W2, np.zeros(N_HIDDEN), W3, np.zeros(N_OUT)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def generate(runs, n, order, snapshots, per_snapshot, seed, log=print):
    """Inputs and targets (torch float32 device tensors) from `runs` runs."""
    import torch

    import paper_1211_2205_amd as pa
    import workloads as wl

    rng = np.random.Generator(np.random.PCG64(seed))
    total = runs * snapshots * per_snapshot
    X = torch.empty((total, N_IN), dtype=torch.float32, device="cuda")
    T = torch.empty((total, N_OUT), dtype=torch.float32, device="cuda")
    prob0 = wl.closure_instance(0, order, n)
    s = pa.Solver.from_problem(prob0, precision="fp32")
    steps = s.nsteps
    cuts = [round(steps * (q + 1) / snapshots) for q in range(snapshots)]
    off = 0
    t0 = time.time()
    for r in range(runs):
        if r:
            prob = wl.closure_instance(r, order, n)
            s.set_absorption(prob.sigma_a)
            s.set_scattering(prob.sigma_s0)
            s.set_source(0, prob.source[0])
            s.reset()
        done = 0
        for c in cuts:
            s.advance(c - done)
            done = c
            pts = rng.integers(0, n, size=(per_snapshot, 2)).astype(np.int32)
            s.closure_samples(pts, X[off:off + per_snapshot], T[off:off + per_snapshot])
            off += per_snapshot
        if (r + 1) % 100 == 0 or r + 1 == runs:
            log(f"closure data: {r + 1}/{runs} P_{order} runs, {off} samples, {time.time() - t0:.1f} s")
    s.close()
    return X, T


def generate_loop(params, runs, first, n, order, snapshots, per_snapshot, seed, log=print):
    """Inputs from P_5 + closure states (network `params` as it acts in the
    solver) and targets from the order-`order` run of the same instance at
    the same snapshot fractions of t_final and the same cells: the high-order
    run's order-6 flux F dx / nu_high, rescaled by nu_high / nu_5 to the P_5
    inputs' normalisation."""
    import torch

    import paper_1211_2205_amd as pa
    import workloads as wl

    rng = np.random.Generator(np.random.PCG64(seed))
    total = runs * snapshots * per_snapshot
    X = torch.empty((total, N_IN), dtype=torch.float32, device="cuda")
    T = torch.empty((total, N_OUT), dtype=torch.float32, device="cuda")
    Xh = torch.empty((per_snapshot, N_IN), dtype=torch.float32, device="cuda")
    nu5 = torch.empty(per_snapshot, dtype=torch.float32, device="cuda")
    nuh = torch.empty(per_snapshot, dtype=torch.float32, device="cuda")
    off = 0
    t0 = time.time()
    unstable = 0
    for r in range(first, first + runs):
        hi = pa.Solver.from_problem(wl.closure_instance(r, order, n), precision="fp32")
        lo = pa.Solver.from_problem(wl.closure_instance(r, 5, n), precision="fp32", closure="learned")
        hi.bind_torch()
        lo.bind_torch()
        lo.load_closure(params)
        done_h = done_l = 0
        for q in range(snapshots):
            ch = round(hi.nsteps * (q + 1) / snapshots)
            cl = round(lo.nsteps * (q + 1) / snapshots)
            hi.advance(ch - done_h)
            lo.advance(cl - done_l)
            done_h, done_l = ch, cl
            pts = rng.integers(0, n, size=(per_snapshot, 2)).astype(np.int32)
            sl = slice(off, off + per_snapshot)
            lo.closure_features(pts, X[sl], nu5)
            hi.closure_samples(pts, Xh, T[sl])
            hi.closure_features(pts, Xh, nuh)
            T[sl] *= (nuh / nu5).unsqueeze(1)
            off += per_snapshot
        bad = not bool(torch.isfinite(X[off - snapshots * per_snapshot:off]).all())
        if bad:  # a run that lost finiteness contributes nothing
            unstable += 1
            off -= snapshots * per_snapshot
        hi.close()
        lo.close()
        if (r - first + 1) % 100 == 0:
            log(f"closure loop data: {r - first + 1}/{runs} runs, {off} samples, {time.time() - t0:.1f} s")
    log(f"closure loop data: {runs} runs from instance {first}, {off} samples ({unstable} unstable runs dropped), "
        f"{time.time() - t0:.1f} s")
    return X[:off], T[:off]


def train(X, T, epochs, batch, lr, seed, val_fraction=0.02, log=print, init=None):
    import torch

    import paper_1211_2205_amd as pa

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    n = X.shape[0]
    perm = torch.randperm(n, device="cuda", generator=g)
    nval = max(batch, int(n * val_fraction))
    val, tr = perm[:nval], perm[nval:]
    Xv, Tv = X[val[:batch]].contiguous(), T[val[:batch]].contiguous()
    net = pa.MLP(batch)
    net.set_params(init_params(seed) if init is None else init)
    steps_per_epoch = tr.numel() // batch
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        order = tr[torch.randperm(tr.numel(), device="cuda", generator=g)]
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            x, t = X[idx].contiguous(), T[idx].contiguous()
            rate = lr * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * step / max(1, total))))
            want = (step % 500 == 0) or step == total - 1
            loss = net.train_step(x, t, rate, want_loss=want)
            if want:
                _, vloss = net.gradients(Xv, Tv)
                hist.append({"step": step, "epoch": ep, "lr": rate, "train_loss": loss, "val_loss": vloss})
                log(f"closure train: step {step}/{total} lr {rate:.2e} loss {loss:.4e} val {vloss:.4e} "
                    f"({time.time() - t0:.1f} s)")
            step += 1
    params = net.params()
    net.close()
    return params, hist


def scale_output(params, alpha):
    """The network with its output layer (W3, b3) multiplied by alpha."""
    p = np.array(params, dtype=np.float32, copy=True)
    p[-(N_OUT * N_HIDDEN + N_OUT):] *= np.float32(alpha)
    return p


def calibrate(params, seeds, n, order, alphas, log=print):
    """A-posteriori output scale: the alpha of `alphas` whose P_5 closure
    solutions have the smallest mean relative L2 error of the zeroth moment
    against the order-`order` runs of the given (training) instances; runs
    that lose finiteness or grow beyond ten times the reference are rejected."""
    import paper_1211_2205_amd as pa
    import workloads as wl

    def r00(prob, p=None):
        s = pa.Solver.from_problem(prob, precision="fp32", closure="learned" if p is not None else "pn")
        if p is not None:
            s.load_closure(p)
        s.run()
        out = s.get_moment(0)
        s.close()
        return out

    refs = [r00(wl.closure_instance(k, order, n)) for k in seeds]
    table = []
    for a in alphas:
        p = scale_output(params, a)
        errs = []
        for k, ref in zip(seeds, refs):
            u = r00(wl.closure_instance(k, 5, n), p)
            ok = np.all(np.isfinite(u)) and np.max(np.abs(u)) <= 10 * np.max(np.abs(ref))
            errs.append(math.sqrt(float(np.sum((u - ref) ** 2)) / float(np.sum(ref ** 2))) if ok else math.inf)
        table.append({"alpha": a, "mean_err": float(np.mean(errs))})
        log(f"closure calibrate: alpha {a:.2f} mean R00 error {np.mean(errs):.4e}")
    best = min(table, key=lambda r: r["mean_err"])
    return best["alpha"], table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="parameter blob (.npy)")
    ap.add_argument("--runs", type=int, default=2000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--order", type=int, default=31)
    ap.add_argument("--snapshots", type=int, default=8)
    ap.add_argument("--per-snapshot", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=12112205)
    ap.add_argument("--calibrate-runs", type=int, default=8,
                    help="training instances (indices 0..k-1) for the a-posteriori output scale")
    ap.add_argument("--alphas", default="0.3,0.4,0.5,0.6,0.7,0.8,1.0")
    ap.add_argument("--loop-rounds", type=int, default=4, help="rounds of training on P_5 + closure states")
    ap.add_argument("--loop-runs", type=int, default=400, help="training instances per loop round")
    ap.add_argument("--loop-epochs", type=int, default=3)
    ap.add_argument("--loop-lr", type=float, default=5e-4)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    import torch

    t0 = time.time()
    X, T = generate(args.runs, args.n, args.order, args.snapshots, args.per_snapshot, args.seed, log)
    t1 = time.time()
    params, hist = train(X, T, args.epochs, args.batch, args.lr, args.seed, log=log)
    nsamples = int(X.shape[0])
    t2 = time.time()
    alphas = [float(a) for a in args.alphas.split(",")]
    alpha, table = 1.0, []
    if args.calibrate_runs > 0:
        alpha, table = calibrate(params, range(args.calibrate_runs), args.n, args.order, alphas, log)
    loops = []
    for rnd in range(args.loop_rounds):
        # the network as it acts in the solver (scaled by the current alpha)
        # produces the states; the raw network is trained further on them
        first = args.calibrate_runs + rnd * args.loop_runs
        Xl, Tl = generate_loop(scale_output(params, alpha), args.loop_runs, first, args.n, args.order,
                               args.snapshots, args.per_snapshot, args.seed + 1 + rnd, log)
        X, T = torch.cat([X, Xl]), torch.cat([T, Tl])
        del Xl, Tl
        params, h = train(X, T, args.loop_epochs, args.batch, args.loop_lr, args.seed + 1 + rnd, log=log,
                          init=params)
        a, tab = (calibrate(params, range(args.calibrate_runs), args.n, args.order, alphas, log)
                  if args.calibrate_runs > 0 else (1.0, []))
        loops.append({"round": rnd, "first_instance": first, "samples": int(X.shape[0]), "history": h,
                      "alpha": a, "calibration": tab})
        alpha, table = a, tab
    nsamples = int(X.shape[0])
    del X, T
    t3 = time.time()
    params = scale_output(params, alpha)
    np.save(args.out, params)
    meta = {"runs": args.runs, "n": args.n, "order": args.order, "snapshots": args.snapshots,
            "per_snapshot": args.per_snapshot, "samples": nsamples, "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "seed": args.seed, "data_s": t1 - t0, "train_s": t2 - t1,
            "loop_s": t3 - t2, "history": hist, "loop_rounds": loops, "alpha": alpha, "calibration": table}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"closure train: wrote {args.out} (alpha {alpha}; data {t1 - t0:.1f} s, training {t2 - t1:.1f} s)")


if __name__ == "__main__":
    sys.exit(main())
